"""Pins for the mutual-reachability MST oracle: Kruskal over every pair on tiny
clouds (written here with Python floats), scipy's minimum spanning tree on
the dense mutual-reachability matrix (the weight multiset of every MST is the
same), and scikit-learn's HDBSCAN end to end (points to flat labels)."""
import numpy as np
import pytest

from oracle.emst import core_distances2, emst
from oracle.flat_clusters import decisions_safe, flat_clusters


def cloud(n, dim, seed, kind="normal"):
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.normal(0, 1, (n, dim)).astype(np.float32)
    if kind == "blobs":
        centers = rng.uniform(-20, 20, (5, dim))
        return (centers[rng.integers(0, 5, n)] + rng.normal(0, 1, (n, dim))).astype(np.float32)
    return rng.uniform(0, 1, (n, dim)).astype(np.float32)


def kruskal_reference(x32, min_pts):
    pts = [[float(c) for c in row] for row in np.asarray(x32, np.float32)]
    n = len(pts)

    def d2(i, j):
        acc = 0.0
        for a, b in zip(pts[i], pts[j]):
            t = a - b
            acc = acc + t * t
        return acc
    core = []
    for i in range(n):
        ds = sorted(d2(i, j) for j in range(n) if j != i)
        core.append(0.0 if min_pts == 1 else ds[min_pts - 2])
    keys = sorted((max(core[i], core[j], d2(i, j)), i, j) for i in range(n) for j in range(i + 1, n))
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    out = []
    for k in keys:
        a, b = find(k[1]), find(k[2])
        if a != b:
            parent[a] = b
            out.append(k)
    return out


@pytest.mark.parametrize("seed", range(8))
def test_matches_kruskal_over_every_pair(seed):
    rng = np.random.default_rng(seed)
    for _ in range(6):
        n = int(rng.integers(2, 40))
        dim = int(rng.integers(1, 5))
        min_pts = int(rng.integers(1, min(n, 6) + 1))
        x = cloud(n, dim, int(rng.integers(1 << 30)), ["normal", "blobs", "uniform"][seed % 3])
        if seed % 4 == 3:
            x = np.round(x * 2) / 2          # coarse grid: many equal distances, ties decided by ids
        u, v, w64, w32, mrd2 = emst(x, min_pts)
        ref = kruskal_reference(x, min_pts)
        assert [(float(a), int(b), int(c)) for a, b, c in zip(mrd2, u, v)] == ref
        assert np.array_equal(w64, np.sqrt(mrd2)) and np.array_equal(w32, w64.astype(np.float32))


@pytest.mark.parametrize("min_pts", [1, 2, 5])
def test_weight_multiset_matches_scipy(min_pts):
    from scipy.sparse.csgraph import minimum_spanning_tree
    x = cloud(300, 3, 11 + min_pts, "blobs")
    u, v, w64, _, mrd2 = emst(x, min_pts)
    xd = x.astype(np.float64)
    core = np.sqrt(core_distances2(x, min_pts))
    d = np.sqrt(((xd[:, None, :] - xd[None, :, :]) ** 2).sum(-1))
    mr = np.maximum(np.maximum(d, core[:, None]), core[None, :])
    np.fill_diagonal(mr, 0)
    t = minimum_spanning_tree(mr).tocoo()
    assert t.nnz == len(w64)
    assert np.allclose(np.sort(t.data), np.sort(w64), rtol=1e-12, atol=0)


def test_core_distance_closed_forms():
    x = np.array([[0.0], [1.0], [3.0], [7.0]], np.float32)
    assert list(core_distances2(x, 1)) == [0, 0, 0, 0]
    assert list(core_distances2(x, 2)) == [1, 1, 4, 16]
    assert list(core_distances2(x, 3)) == [9, 4, 9, 36]
    u, v, w64, w32, mrd2 = emst(x, 1)                 # a line: consecutive points, by length
    assert list(zip(u, v)) == [(0, 1), (1, 2), (2, 3)] and list(w64) == [1, 2, 4]
    with pytest.raises(ValueError):
        core_distances2(x, 5)


@pytest.mark.parametrize("seed,mcs", [(1, 10), (2, 15), (3, 25), (4, 8)])
def test_end_to_end_matches_sklearn_hdbscan(seed, mcs):
    """min_pts = 2 (mutual reachability of tree edges is then the plain
    distance, so the weights are tie-free); larger min_pts share core
    distances between edges, and the order of such tied merges is an
    implementation choice, so only the MST itself is pinned there (by the
    Kruskal reference above)."""
    from sklearn.cluster import HDBSCAN
    min_pts = 2
    x = cloud(600, 2 + seed % 2, seed, "blobs")
    u, v, w64, w32, _ = emst(x, min_pts)
    if len(np.unique(w32)) != len(w32):
        pytest.skip("tied weights: the single-linkage order is not unique")
    lab, st, info = flat_clusters(len(x), u, v, w32, mcs, return_info=True)
    assert decisions_safe(info)
    h = HDBSCAN(min_cluster_size=mcs, min_samples=min_pts, allow_single_cluster=False).fit(x.astype(np.float64))

    def canon(a):
        names, out = {}, []
        for z in a:
            out.append(-1 if z < 0 else names.setdefault(int(z), len(names)))
        return np.array(out)
    assert np.array_equal(canon(lab), canon(h.labels_))
    assert st.size >= 2
