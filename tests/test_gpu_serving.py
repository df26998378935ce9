"""Continuous-batching server: every request's dendrogram is the same as when it
is built alone, the byte budget is never exceeded, and batches overlap."""
import time

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    pd.library()
    yield


def test_server_results_match_alone_and_budget_holds():
    import paper_2401_06089_amd as pd
    from paper_2401_06089_amd.serve import DendrogramServer, Request, request_footprint, slot_bytes

    dev = torch.device("cuda:0")
    sizes = np.floor(np.exp(np.log(1e3) + gen.uniform_f64(24, 7, 30) * (np.log(3e5) - np.log(1e3))))
    pool = []
    for i, n in enumerate(sizes.astype(np.int64)):
        t = gen.rrt(int(n), 100 + i, weights="lognormal") if i % 2 else gen.caterpillar(int(n), None, 1e-3, i)
        pool.append((t, tuple(torch.from_numpy(a).to(dev) for a in (t.u, t.v, t.w))))
    alone = []
    for t, (u, v, w) in pool:
        ep, vp = pd.dendrogram(u, v, w, n=t.n)
        alone.append((ep.cpu().numpy(), vp.cpu().numpy()))
    # every pool tree, built alone, is the oracle's dendrogram; so then is
    # every result in the mix that equals it
    for k, (t, _) in enumerate(pool):
        oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
        assert np.array_equal(alone[k][0], oep) and np.array_equal(alone[k][1], ovp), f"pool tree {k}"

    # three slots sized for 600,000-edge batches, plus room for the outputs of
    # about three of the largest requests: admission has to wait for bytes
    biggest = int(sizes.max())
    reserved = 3 * slot_bytes(max(600_000, biggest - 1), 4096)
    budget = reserved + 3 * request_footprint(biggest)
    srv = DendrogramServer(budget, streams=3, max_batch_edges=600_000, max_tree_vertices=biggest)
    assert srv.reserved == reserved
    picks = (gen.uniform_f64(160, 8, 31) * len(pool)).astype(np.int64)
    reqs = []
    t0 = time.perf_counter()
    for i, p in enumerate(picks):
        t, (u, v, w) = pool[int(p)]
        r = Request(i, t.n, u, v, w, arrival=time.perf_counter())
        reqs.append((int(p), r))
        srv.submit(r)
        if i % 40 == 39:
            time.sleep(0.002)
    for p, r in reqs:
        ep, vp = r.future.result(timeout=120)
        assert np.array_equal(ep.cpu().numpy(), alone[p][0]), f"request {r.rid} differs in the mix"
        assert np.array_equal(vp.cpu().numpy(), alone[p][1])
    srv.close()
    assert srv.peak_in_use <= budget
    assert srv.batches < len(reqs)            # requests were batched together
    assert srv.max_concurrent >= 2            # batches ran side by side on different streams
    assert time.perf_counter() - t0 < 120


def test_server_rejects_oversized_requests():
    from paper_2401_06089_amd.serve import DendrogramServer, Request, slot_bytes
    t = gen.rrt(100_000, 1)
    u, v, w = (torch.from_numpy(a).cuda() for a in (t.u, t.v, t.w))
    # the tree is larger than the slots were sized for
    srv = DendrogramServer(slot_bytes(1000, 8) + (1 << 20), streams=1, max_batch_edges=1000, max_batch_trees=8,
                           max_tree_vertices=1001)
    r = Request(0, t.n, u, v, w, arrival=time.perf_counter())
    srv.submit(r)
    with pytest.raises(MemoryError):
        r.future.result(timeout=10)
    srv.close()
    # its outputs do not fit the budget left after the slots' reservation
    srv = DendrogramServer(slot_bytes(200_000, 8) + 1000, streams=1, max_batch_edges=200_000, max_batch_trees=8,
                           max_tree_vertices=200_001)
    r = Request(1, t.n, u, v, w, arrival=time.perf_counter())
    srv.submit(r)
    with pytest.raises(MemoryError):
        r.future.result(timeout=10)
    srv.close()
    # slots that do not fit the budget at all
    with pytest.raises(ValueError):
        DendrogramServer(1 << 20, streams=1)


def test_server_reports_an_input_error_on_its_request_only():
    """A NaN weight in one tree of a batch: that request fails with
    NAN_WEIGHT, the others of the same batch still get the oracle's result."""
    import paper_2401_06089_amd as pd
    from paper_2401_06089_amd.serve import DendrogramServer, Request, slot_bytes
    dev = torch.device("cuda:0")
    trees = [gen.rrt(2_000 + 300 * k, 40 + k) for k in range(6)]
    bad = 3
    reqs = []
    srv = DendrogramServer(slot_bytes(100_000, 64) + (1 << 24), streams=1, max_batch_edges=100_000,
                           max_batch_trees=64, max_tree_vertices=100_001)
    with srv.cv:                       # hold the dispatcher so that all six form one batch
        for k, t in enumerate(trees):
            w = t.w.copy()
            if k == bad:
                w[7] = np.float32("nan")
            r = Request(k, t.n, *(torch.from_numpy(a).to(dev) for a in (t.u, t.v, w)), arrival=time.perf_counter())
            reqs.append(r)
            srv.submit(r)
    for k, r in enumerate(reqs):
        if k == bad:
            with pytest.raises(pd.PandoraError) as ei:
                r.future.result(timeout=60)
            assert ei.value.status == pd.NAN_WEIGHT
        else:
            ep, vp = r.future.result(timeout=60)
            oep, ovp = oracle.dendrogram(trees[k].n, trees[k].u, trees[k].v, trees[k].w)
            assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)
    srv.close()


def test_server_waits_for_inputs_still_being_written():
    """A client writes a request's weights on its own stream, behind a long
    GPU spin, and submits at once: the worker's stream must wait for that
    write (the event recorded at submit), so the result is still the
    oracle's."""
    from paper_2401_06089_amd.serve import DendrogramServer, Request

    dev = torch.device("cuda:0")
    t = gen.rrt(200_000, 5, weights="lognormal")
    u = torch.from_numpy(t.u).to(dev)
    v = torch.from_numpy(t.v).to(dev)
    w_host = torch.from_numpy(t.w).pin_memory()
    srv = DendrogramServer(1 << 36, streams=2)
    client = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(client):
        w = torch.zeros(t.n - 1, dtype=torch.float32, device=dev)   # wrong until the copy lands
        torch.cuda._sleep(200_000_000)                               # on the order of 0.1 s of spinning
        w.copy_(w_host, non_blocking=True)
        r = Request(0, t.n, u, v, w, arrival=time.perf_counter())
        srv.submit(r)
    ep, vp = r.future.result(timeout=120)
    srv.close()
    oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)
