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
    from paper_2401_06089_amd.serve import DendrogramServer, Request, request_footprint

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

    budget = 3 * max(request_footprint(int(n)) for n in sizes)   # forces admission waits
    srv = DendrogramServer(budget, streams=3, max_batch_edges=600_000)
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


def test_server_rejects_oversized_request():
    from paper_2401_06089_amd.serve import DendrogramServer, Request
    t = gen.rrt(100_000, 1)
    u, v, w = (torch.from_numpy(a).cuda() for a in (t.u, t.v, t.w))
    srv = DendrogramServer(1 << 20, streams=1)
    r = Request(0, t.n, u, v, w, arrival=time.perf_counter())
    srv.submit(r)
    with pytest.raises(MemoryError):
        r.future.result(timeout=10)
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
