"""Captured calls (HIP graphs): every replay, with eager library work and
synchronisations in between, matches the eager call and the oracle."""
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


@pytest.mark.parametrize("n", [2, 4097, 100_000, 1_000_000])
def test_graph_replays_match_eager_and_oracle(n):
    import paper_2401_06089_amd as pd
    trees = [gen.rrt(n, 11), gen.shuffled(gen.pref_attach(n, 12), 12), gen.caterpillar(n, None, 1e-3, 13)]
    dev = torch.device("cuda:0")
    t0 = trees[0]
    u = torch.from_numpy(t0.u).to(dev)
    v = torch.from_numpy(t0.v).to(dev)
    w = torch.from_numpy(t0.w).to(dev)
    g = pd.Graph(u, v, w)
    for rep in range(6):
        t = trees[rep % 3]
        u.copy_(torch.from_numpy(t.u))       # new inputs, same buffers
        v.copy_(torch.from_numpy(t.v))
        w.copy_(torch.from_numpy(t.w))
        ep, vp = g.launch()
        ep, vp = ep.cpu().numpy(), vp.cpu().numpy()
        eep, evp = pd.dendrogram(u, v, w)      # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(ep, eep.cpu().numpy()) and np.array_equal(vp, evp.cpu().numpy())
        if rep < 3:
            oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
            assert np.array_equal(ep, oep) and np.array_equal(vp, ovp)
    assert pd.last_stats()["sync_free"] in (0, 1)
    g.close()


def test_graph_batched_and_errors():
    import paper_2401_06089_amd as pd
    trees = [gen.rrt(s, s) for s in (1, 2, 3000, 17, 50_000)]
    f = gen.forest_from_trees(trees)
    u, v, w = (torch.from_numpy(a).cuda() for a in (f.u, f.v, f.w))
    g = pd.Graph(u, v, w, voff=f.voff)
    oep, ovp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
    for _ in range(3):
        ep, vp = g.launch()
        assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)
    bad = f.u.copy()
    bad[10] = 10**6
    u.copy_(torch.from_numpy(bad))
    with pytest.raises(pd.PandoraError) as e:
        g.launch()
    assert e.value.status == pd.BAD_VERTEX
    u.copy_(torch.from_numpy(f.u))
    ep, vp = g.launch()                       # recovers on the next replay
    assert np.array_equal(ep.cpu().numpy(), oep)
    g.close()
