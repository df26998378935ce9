"""Stream-ordered calls, deferred status and caller-owned scratch: every
result equals the synchronous call's (and the oracle's), input errors surface
through the stream's status word, and a caller's buffer serves as scratch."""
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


def dev_tree(t):
    return tuple(torch.from_numpy(a).cuda() for a in (t.u, t.v, t.w))


def test_async_matches_sync_across_sizes_and_scratch_growth():
    import paper_2401_06089_amd as pd
    s = torch.cuda.Stream()
    trees = [gen.rrt(2, 1), gen.rrt(3000, 2), gen.rrt(40_000, 3), gen.shuffled(gen.pref_attach(300_000, 4), 4),
             gen.caterpillar(1_000_000, None, 1e-3, 5), gen.rrt(5000, 6)]
    outs = []
    with torch.cuda.stream(s):
        for t in trees:                      # scratch grows twice on the way
            u, v, w = dev_tree(t)
            outs.append(pd.dendrogram_async(u, v, w, stream=s))
    assert pd.stream_status(s) == pd.OK
    for t, (ep, vp) in zip(trees, outs):
        oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
        assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)


def test_async_single_vertex_and_forest_of_singletons():
    import paper_2401_06089_amd as pd
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    ep, vp = pd.dendrogram_async(e, e, torch.empty(0, dtype=torch.float32, device="cuda"), n=1)
    assert pd.stream_status() == pd.OK
    assert vp.cpu().tolist() == [-1]
    ep, vp = pd.dendrogram_batched_async(np.arange(6, dtype=np.int64), e, e,
                                         torch.empty(0, dtype=torch.float32, device="cuda"))
    assert pd.stream_status() == pd.OK
    assert vp.cpu().tolist() == [-1] * 5


def test_deferred_errors_are_reported_merged_and_cleared():
    import paper_2401_06089_amd as pd
    base = gen.rrt(50_000, 9)
    s = torch.cuda.Stream()

    def call(kind):
        t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w.copy())
        if kind == "cycle":
            t.u[700], t.v[700] = t.u[800], t.v[800]
        elif kind == "bad":
            t.v[5] = base.n + 3
        elif kind == "nan":
            t.w[17] = np.float32("nan")
        u, v, w = dev_tree(t)
        with torch.cuda.stream(s):
            return pd.dendrogram_async(u, v, w, stream=s)

    call("cycle")
    assert pd.stream_status(s) == pd.NOT_A_TREE
    assert pd.stream_status(s) == pd.OK               # read once, then cleared
    call("nan")
    assert pd.stream_status(s) == pd.NAN_WEIGHT
    call("cycle")
    call("bad")
    call("ok")
    assert pd.stream_status(s) == pd.BAD_VERTEX       # merged: the most specific wins
    ep, vp = call("ok")                               # the stream recovers
    assert pd.stream_status(s) == pd.OK
    oep, ovp = oracle.dendrogram(base.n, base.u, base.v, base.w)
    assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)


def test_batched_async_reuses_staging_in_stream_order():
    import paper_2401_06089_amd as pd
    s = torch.cuda.Stream()
    forests, outs = [], []
    with torch.cuda.stream(s):
        for k in range(9):                   # more calls than staging slots, all queued at once
            sizes = [int(x) for x in 2 + (gen.uniform_f64(30 + k, 40 + k, 3) * 20_000)]
            f = gen.forest_from_trees([gen.rrt(n, 100 * k + i) for i, n in enumerate(sizes)])
            u, v, w = dev_tree(f)
            forests.append(f)
            outs.append(pd.dendrogram_batched_async(f.voff, u, v, w, stream=s))
    assert pd.stream_status(s) == pd.OK
    for f, (ep, vp) in zip(forests, outs):
        oep, ovp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
        assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)


def test_caller_owned_workspace():
    import paper_2401_06089_amd as pd
    t = gen.shuffled(gen.rrt(200_000, 11), 11)
    u, v, w = dev_tree(t)
    oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    s = torch.cuda.Stream()
    need = pd.workspace_bytes(t.n)
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert buf.data_ptr() % 256 == 0
    try:
        pd.set_workspace(buf, stream=s)
        with torch.cuda.stream(s):
            ep, vp = pd.dendrogram(u, v, w, stream=s)
            ep2, vp2 = pd.dendrogram_async(u, v, w, stream=s)
        assert pd.stream_status(s) == pd.OK
        for a, b in ((ep, oep), (vp, ovp), (ep2, oep), (vp2, ovp)):
            assert np.array_equal(a.cpu().numpy(), b)
        big = gen.rrt(400_000, 12)
        bu, bv, bw = dev_tree(big)
        with pytest.raises(pd.PandoraError) as ei:          # more than the caller's buffer holds
            with torch.cuda.stream(s):
                pd.dendrogram(bu, bv, bw, stream=s)
        assert ei.value.status == pd.OUT_OF_MEMORY
    finally:
        pd.set_workspace(None, stream=s)
    with torch.cuda.stream(s):                                # library-owned scratch again
        ep, vp = pd.dendrogram(u, v, w, stream=s)
    assert np.array_equal(ep.cpu().numpy(), oep)
