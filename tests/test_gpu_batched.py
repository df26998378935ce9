"""Batched forests (many trees in one call): bit-exact with the oracle, and each
tree's slice identical to the same tree built alone."""
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


def _run_forest(f):
    import paper_2401_06089_amd as pd
    u, v, w = (torch.from_numpy(a).cuda() for a in (f.u, f.v, f.w))
    ep, vp = pd.dendrogram_batched(f.voff, u, v, w)
    torch.cuda.synchronize()
    return ep.cpu().numpy(), vp.cpu().numpy()


def _check_forest(f, tag):
    ep, vp = _run_forest(f)
    oep, ovp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
    assert np.array_equal(vp, ovp), f"{tag}: vertex_parent differs at {np.flatnonzero(vp != ovp)[:5]}"
    assert np.array_equal(ep, oep), f"{tag}: edge_parent differs at {np.flatnonzero(ep != oep)[:5]}"
    return ep, vp


def test_forest_small_mixed_shapes():
    trees = []
    for s in range(60):
        n = int(gen.uniform_f64(1, s, 20)[0] * 20000) + 1
        k = s % 4
        t = (gen.rrt(n, s) if k == 0 else gen.caterpillar(n, None, 1e-3, s) if k == 1
             else gen.shuffled(gen.pref_attach(n, s), s) if k == 2 else gen.path_mono(n))
        trees.append(t)
    _check_forest(gen.forest_from_trees(trees), "mixed")


def test_forest_many_single_vertices_and_one_big_tree():
    one = gen.Tree(1, np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float32))
    trees = [one] * 9000 + [gen.rrt(3000, 1)] + [one] * 50
    _check_forest(gen.forest_from_trees(trees), "singletons")


def test_forest_many_equal_tiny_trees():
    """Thousands of components finish at the same level (more than the LDS tail
    holds as vertices)."""
    trees = [gen.path_mono(3) for _ in range(12000)] + [gen.rrt(10, s) for s in range(3000)]
    _check_forest(gen.forest_from_trees(trees), "tiny")


def test_forest_slices_equal_standalone_calls():
    import paper_2401_06089_amd as pd
    f = gen.c4_batched(3, B=200, target_edges=2_000_000, hi=200_000)
    ep, vp = _check_forest(f, "c4-small")
    for b in range(0, f.B, 17):
        t = f.tree(b)
        u, v, w = (torch.from_numpy(a).cuda() for a in (t.u, t.v, t.w))
        sep, svp = pd.dendrogram(u, v, w, n=t.n)
        v0, v1 = int(f.voff[b]), int(f.voff[b + 1])
        assert np.array_equal(svp.cpu().numpy(), vp[v0:v1])
        assert np.array_equal(sep.cpu().numpy(), ep[v0 - b:v1 - b - 1])


def test_forest_error_in_one_tree():
    import paper_2401_06089_amd as pd
    trees = [gen.rrt(1000, s) for s in range(5)]
    trees[3].u[10] = 5000                     # outside tree 3's [0, 1000)
    f = gen.forest_from_trees(trees)
    with pytest.raises(pd.PandoraError) as e:
        _run_forest(f)
    assert e.value.status == pd.BAD_VERTEX


def test_forest_full_c4():
    f = gen.c4_batched(0)
    assert f.B == 4096 and abs(f.m_total - 50_000_000) < 600_000
    _check_forest(f, "c4")
