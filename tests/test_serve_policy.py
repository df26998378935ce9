"""Admission and batching policy of the dendrogram server, on the CPU: a
server with no worker streams, whose batch selection is called directly.
Requests carry no tensors here; only their sizes matter to the policy."""
import pytest

from paper_2401_06089_amd.serve import DendrogramServer, Request, request_footprint


def make(sizes, budget, cap, policy):
    srv = DendrogramServer(budget, streams=0, max_batch_edges=cap, policy=policy)
    reqs = []
    for i, n in enumerate(sizes):
        r = Request(i, n, None, None, None, arrival=float(i))
        srv.submit(r)
        reqs.append(r)
    return srv, reqs


def take(srv):
    with srv.cv:
        b = srv._take_batch()
    return [r.rid for r in b] if b else None


def test_footprint_is_the_outputs():
    f = [request_footprint(n) for n in (10, 1000, 100_000, 10_000_000)]
    assert all(a < b for a, b in zip(f, f[1:]))
    assert f[-1] == 4 * (10_000_000 - 1) + 4 * 10_000_000    # edge_parent + vertex_parent


def test_tree_cap_limits_a_batch():
    srv = DendrogramServer(10**12, streams=0, max_batch_edges=10**9, max_batch_trees=3, policy="fifo")
    for i in range(7):
        srv.submit(Request(i, 100, None, None, None, arrival=float(i)))
    assert take(srv) == [0, 1, 2]
    assert take(srv) == [3, 4, 5]
    assert take(srv) == [6]


def test_tree_larger_than_the_slots_is_rejected_at_submit():
    srv = DendrogramServer(10**12, streams=0, max_tree_vertices=1000)
    r = Request(0, 1001, None, None, None, arrival=0.0)
    srv.submit(r)
    with pytest.raises(MemoryError):
        r.future.result(timeout=1)
    assert take(srv) is None


def test_fifo_takes_arrival_order_up_to_the_edge_cap():
    srv, _ = make([1000, 2000, 500_000, 10], budget=10**12, cap=400_000, policy="fifo")
    assert take(srv) == [0, 1]           # the 500k request would pass the cap: stop there
    assert take(srv) == [2]              # a lone request may exceed the cap
    assert take(srv) == [3]
    assert take(srv) is None


def test_small_first_fills_around_a_large_request():
    srv, _ = make([1000, 2000, 500_000, 10, 300], budget=10**12, cap=400_000, policy="small_first")
    assert take(srv) == [0, 3, 4, 1]     # oldest first, then the smallest that fit
    assert take(srv) == [2]


def test_small_first_never_starves_the_oldest():
    srv, _ = make([900_000, 10, 20, 30], budget=10**12, cap=100, policy="small_first")
    assert take(srv) == [0]              # the oldest heads the batch even when it is the largest
    assert take(srv) == [1, 2, 3]


@pytest.mark.parametrize("policy", ["fifo", "small_first"])
def test_budget_is_never_exceeded(policy):
    sizes = [200_000, 150_000, 100_000, 50_000, 25_000]
    budget = request_footprint(200_000) + request_footprint(50_000)
    srv, reqs = make(sizes, budget=budget, cap=10**9, policy=policy)
    first = take(srv)
    assert sum(reqs[i].footprint for i in first) <= budget
    assert srv.in_use <= budget and srv.peak_in_use <= budget
    assert 0 in first
    take(srv)                            # whatever else is admitted still fits the budget
    assert srv.in_use <= budget and srv.peak_in_use <= budget


def test_oversized_request_is_rejected_at_submit():
    srv = DendrogramServer(1 << 20, streams=0)
    r = Request(0, 1_000_000, None, None, None, arrival=0.0)
    srv.submit(r)
    with pytest.raises(MemoryError):
        r.future.result(timeout=1)
    assert take(srv) is None


def test_unknown_policy():
    with pytest.raises(ValueError):
        DendrogramServer(1 << 30, streams=0, policy="lifo")


def test_submit_after_close_fails_the_request():
    srv = DendrogramServer(10**12, streams=0)
    srv.close()
    r = Request(0, 100, None, None, None, arrival=0.0)
    srv.submit(r)
    with pytest.raises(RuntimeError):
        r.future.result(timeout=1)
