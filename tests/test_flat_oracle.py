"""Pins for the flat-cluster oracle (HDBSCAN* excess-of-mass clusters from
the dendrogram): the component-removal brute force on tiny trees (bit-equal
stabilities and labels, including exact ties), scikit-learn's HDBSCAN on the
tree's path-maximum distances, and closed forms."""
import numpy as np
import pytest

import gen
from checks import brute_flat_clusters
from oracle.flat_clusters import decisions_safe, flat_clusters


def random_tree(rng, n):
    par = [int(rng.integers(0, i)) for i in range(1, n)]
    perm = rng.permutation(n).astype(np.int32)          # shuffle vertex names
    u = perm[np.arange(1, n)]
    v = perm[np.array(par, dtype=np.int64)] if n > 1 else np.empty(0, np.int32)
    return np.ascontiguousarray(u, np.int32), np.ascontiguousarray(v, np.int32)


@pytest.mark.parametrize("seed", range(6))
def test_matches_brute_force_lognormal(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(40):
        n = int(rng.integers(2, 45))
        mcs = int(rng.integers(2, 9))
        u, v = random_tree(rng, n)
        w = rng.lognormal(0, 1.5, n - 1).astype(np.float32)
        lab, st, info = flat_clusters(n, u, v, w, mcs, return_info=True)
        blab, bst = brute_flat_clusters(n, u, v, w, mcs)
        assert np.array_equal(st, bst)                   # exactly rounded sums of the same terms
        if decisions_safe(info):
            assert np.array_equal(lab, blab), (n, mcs)


@pytest.mark.parametrize("seed", range(4))
def test_matches_brute_force_with_exact_ties(seed):
    """Dyadic weights make every stability an exact small dyadic number, so
    ties between a cluster and its children are exact on both sides and the
    tie rule (the parent wins) is what is tested."""
    rng = np.random.default_rng(200 + seed)
    ties = 0
    for _ in range(400):
        n = int(rng.integers(4, 30))
        mcs = int(rng.integers(2, 5))
        u, v = random_tree(rng, n)
        w = (2.0 ** rng.integers(-1, 2, n - 1)).astype(np.float32)
        lab, st, info = flat_clusters(n, u, v, w, mcs, return_info=True)
        blab, bst = brute_flat_clusters(n, u, v, w, mcs)
        assert np.array_equal(st, bst) and np.array_equal(lab, blab), (n, mcs, w)
        ties += sum(1 for _, s, cs, _b in info["decisions"] if s == cs)
    assert ties > 0


def _path_max(n, u, v, w):
    adj = [[] for _ in range(n)]
    for e in range(n - 1):
        adj[int(u[e])].append((int(v[e]), float(w[e])))
        adj[int(v[e])].append((int(u[e]), float(w[e])))
    D = np.zeros((n, n))
    for s in range(n):
        stack, seen = [(s, 0.0)], {s}
        while stack:
            x, mx = stack.pop()
            D[s, x] = mx
            for y, wy in adj[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append((y, max(mx, wy)))
    return D


def _canon(lab):
    names, out = {}, []
    for x in lab:
        out.append(-1 if x < 0 else names.setdefault(int(x), len(names)))
    return np.array(out)


@pytest.mark.parametrize("seed", range(5))
def test_matches_sklearn_hdbscan(seed):
    """scikit-learn's HDBSCAN (min_samples=1, so mutual reachability is the
    plain distance) on the subdominant ultrametric of the tree builds the same
    single-linkage hierarchy; with tie-free weights its excess-of-mass labels
    must equal ours up to renaming."""
    from sklearn.cluster import HDBSCAN
    rng = np.random.default_rng(300 + seed)
    clusters = 0
    for _ in range(8):
        n = int(rng.integers(20, 250))
        mcs = int(rng.integers(2, 15))
        t = gen.rrt(n, int(rng.integers(1 << 30)))
        w = rng.lognormal(0, 1.5, n - 1).astype(np.float32)
        if len(np.unique(w)) != n - 1:      # the comparison needs tie-free weights
            continue
        lab, st, info = flat_clusters(n, t.u, t.v, w, mcs, return_info=True)
        if not decisions_safe(info):
            continue
        h = HDBSCAN(min_cluster_size=mcs, min_samples=1, metric="precomputed",
                    allow_single_cluster=False).fit(_path_max(n, t.u, t.v, w))
        assert np.array_equal(_canon(lab), _canon(h.labels_)), (n, mcs)
        clusters += len(st)
    assert clusters > 0


def test_too_small_for_a_split_is_all_noise():
    t = gen.rrt(20, 1)
    lab, st = flat_clusters(t.n, t.u, t.v, t.w + np.float32(0.01), 11)   # n < 2 * mcs
    assert (lab == -1).all() and st.size == 0
    lab, st = flat_clusters(1, np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float32), 2)
    assert list(lab) == [-1] and st.size == 0


def test_two_stars_joined_by_a_bridge():
    """Two stars of s leaves with light spokes, centres joined by a heavy
    edge: each star's dendrogram is a chain, so each star is one leaf cluster
    of the single true split, and both are chosen.  Every spoke removal cuts
    off parts smaller than mcs, so every vertex of a star leaves its cluster
    at 1/a, and a star born at 1/B has stability (s + 1) * (1/a - 1/B)."""
    s, a, B = 9, 0.5, 8.0
    u, v, w = [], [], []
    for c, base in ((0, 1), (s + 1, s + 2)):
        for k in range(s):
            u.append(c)
            v.append(base + k)
            w.append(a)
    u.append(0)
    v.append(s + 1)
    w.append(B)
    n = 2 * (s + 1)
    lab, st = flat_clusters(n, np.array(u, np.int32), np.array(v, np.int32), np.array(w, np.float32), 3)
    assert list(lab) == [0] * (s + 1) + [1] * (s + 1)
    assert np.allclose(st, (s + 1) * (1 / a - 1 / B))


def test_infinite_weight_is_lambda_zero_and_bad_weights_are_rejected():
    t = gen.rrt(50, 3)
    w = t.w + np.float32(0.01)
    w[10] = np.float32("inf")
    lab, st, info = flat_clusters(t.n, t.u, t.v, w, 4, return_info=True)
    blab, bst = brute_flat_clusters(t.n, t.u, t.v, w, 4)
    assert np.array_equal(st, bst)
    if decisions_safe(info):
        assert np.array_equal(lab, blab)
    for bad in (0.0, -1.0, float("nan")):
        w2 = w.copy()
        w2[3] = bad
        with pytest.raises(ValueError):
            flat_clusters(t.n, t.u, t.v, w2, 4)
    with pytest.raises(ValueError):
        flat_clusters(t.n, t.u, t.v, w, 1)


@pytest.mark.parametrize("maker,mcs", [
    (lambda: gen.rrt(20_000, 4, weights="lognormal"), 10),
    (lambda: gen.shuffled(gen.pref_attach(20_000, 5), 5), 25),
    (lambda: gen.caterpillar(20_000, None, 1e-3, 6), 5),
])
def test_midsize_invariants(maker, mcs):
    """Every chosen cluster holds at least mcs vertices, its stability is
    positive, and the chosen clusters are disjoint by construction; labels
    are numbered by smallest vertex id."""
    t = maker()
    w = np.maximum(t.w, np.float32(1e-6))
    lab, st, info = flat_clusters(t.n, t.u, t.v, w, mcs, return_info=True)
    k = st.size
    counts = np.bincount(lab[lab >= 0], minlength=k)
    assert (counts >= mcs).all()
    assert (st > 0).all()
    firsts = [int(np.argmax(lab == c)) for c in range(k)]
    assert firsts == sorted(firsts)
