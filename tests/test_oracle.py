"""Pins for the CPU oracle (no GPU).  Each test checks the oracle against something
other than itself: brute force, exhaustive enumeration, closed forms from the
paper, a library routine, or the paper's structural theorems."""
import itertools

import numpy as np
import pytest

import gen
import oracle
from checks import brute_force, children_sets, invariants, prufer_trees, scipy_merges


def _run(t):
    return oracle.dendrogram(t.n, t.u, t.v, t.w)


# ---- ordering step (Section 3.1.1: sort by weight, consistent tie order) ----

def test_edge_order_matches_lexsort():
    rng = np.random.default_rng(1)
    w = rng.integers(0, 50, 5000).astype(np.float32)          # many ties
    w[::7] = -0.0
    w[::11] = 0.0
    w[3] = np.inf
    w[4] = -np.inf
    got = oracle.edge_order(w)
    # library routine: stable lexicographic sort on (w, id); -0.0 == +0.0
    want = np.lexsort((np.arange(len(w)), w.astype(np.float64) + 0.0))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("threads", [2, 3, 8, 16])
@pytest.mark.parametrize("m", [0, 1, 4097, 50_000, 300_001])
def test_threaded_edge_order_matches_lexsort(m, threads):
    # the merge of sorted runs on several threads gives the same total order
    rng = np.random.default_rng(m + threads)
    w = (rng.integers(0, 40, m).astype(np.float32) - 20) * np.float32(0.25)   # many ties, both signs
    if m > 4:
        w[:4] = [-0.0, 0.0, np.inf, -np.inf]
    want = np.lexsort((np.arange(m), w.astype(np.float64) + 0.0))
    assert np.array_equal(oracle.edge_order(w, threads=threads), want)


@pytest.mark.parametrize("threads", [1, 4])
def test_timed_dendrogram_equals_plain_and_brute_force(threads):
    for seed in range(6):
        t = gen.shuffled(gen.rrt(30, seed), seed)
        t.w[:] = np.random.default_rng(seed).integers(0, 4, 29).astype(np.float32)   # ties
        ep, vp, ts, tw = oracle.dendrogram_timed(t.n, t.u, t.v, t.w, threads=threads)
        bep, bvp = brute_force(t.n, t.u, t.v, t.w)
        assert np.array_equal(ep, bep) and np.array_equal(vp, bvp)
        assert ts >= 0.0 and tw >= 0.0
    t = gen.c1_rrt(0)
    ep, vp, _, _ = oracle.dendrogram_timed(t.n, t.u, t.v, t.w, threads=threads)
    pep, pvp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    assert np.array_equal(ep, pep) and np.array_equal(vp, pvp)


def test_signed_zero_ties_fall_to_id():
    w = np.array([0.0, -0.0, 0.0, -0.0], np.float32)
    assert list(oracle.edge_order(w)) == [0, 1, 2, 3]


# ---- brute force: components at every threshold ----

@pytest.mark.parametrize("seed", range(40))
def test_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    shape = seed % 4
    if shape == 0:
        t = gen.rrt(n, seed)
    elif shape == 1:
        t = gen.shuffled(gen.pref_attach(n, seed), seed)
    elif shape == 2:
        t = gen.shuffled(gen.caterpillar(n, None, 1e-1, seed), seed)
    else:
        t = gen.shuffled(gen.rrt(n, seed), seed)
        t.w[:] = rng.integers(0, 3, n - 1).astype(np.float32)  # heavy ties
    ep, vp = _run(t)
    bep, bvp = brute_force(t.n, t.u, t.v, t.w)
    assert np.array_equal(ep, bep)
    assert np.array_equal(vp, bvp)


def test_exhaustive_small_trees():
    """Every labelled tree on n <= 5 vertices, every weight order and every
    0/1 weight pattern (forced ties); n = 6 with sampled orders and patterns."""
    count = 0
    rng = np.random.default_rng(7)
    for n in range(2, 7):
        for edges in prufer_trees(n):
            u = np.array([e[0] for e in edges], np.int32)
            v = np.array([e[1] for e in edges], np.int32)
            if n <= 5:
                weights = [np.array(p, np.float32) for p in itertools.permutations(range(n - 1))]
                weights += [np.array(b, np.float32) for b in itertools.product([0, 1], repeat=n - 1)]
            else:
                weights = [rng.permutation(n - 1).astype(np.float32) for _ in range(2)]
                weights += [rng.integers(0, 2, n - 1).astype(np.float32) for _ in range(2)]
            for w in weights:
                ep, vp = oracle.dendrogram(n, u, v, w)
                bep, bvp = brute_force(n, u, v, w)
                assert np.array_equal(ep, bep) and np.array_equal(vp, bvp), (edges, w)
                count += 1
    assert count > 8000


# ---- closed forms ----

def test_single_vertex_and_single_edge():
    ep, vp = oracle.dendrogram(1, np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float32))
    assert ep.shape == (0,) and list(vp) == [-1]
    ep, vp = oracle.dendrogram(2, np.array([1], np.int32), np.array([0], np.int32), np.array([0.5], np.float32))
    assert list(ep) == [-1] and list(vp) == [0, 0]


@pytest.mark.parametrize("n", [3, 17, 1000, 20001])
def test_star_is_sorted_chain(n):
    """Theorem lowerbound: the dendrogram of a star is one chain in weight order."""
    t = gen.star(n, seed=n)
    t.w[: (n - 1) // 3] = 0.25       # ties resolved by id
    ep, vp = _run(t)
    order = np.lexsort((np.arange(n - 1), t.w))
    want = np.full(n - 1, -1, np.int32)
    want[order[:-1]] = order[1:]
    assert np.array_equal(ep, want)
    assert vp[0] == order[0]                       # centre: lightest edge
    assert np.array_equal(vp[1:], np.arange(n - 1))  # leaf i: its only edge i-1


@pytest.mark.parametrize("n", [2, 3, 50, 100000])
def test_monotone_path_is_chain(n):
    t = gen.path_mono(n)
    ep, vp = _run(t)
    want = np.arange(1, n, dtype=np.int32)
    want[-1] = -1
    assert np.array_equal(ep, want)
    assert vp[0] == 0 and np.array_equal(vp[1:], np.arange(n - 1))


def test_constant_weights_order_by_id():
    """All weights equal: the order is the id order, so the result equals that
    of strictly increasing weights w = id."""
    t = gen.shuffled(gen.rrt(3000, 5), 5)
    t.w[:] = 1.0
    ep, vp = _run(t)
    t2 = gen.Tree(t.n, t.u, t.v, np.arange(t.m, dtype=np.float32))
    ep2, vp2 = _run(t2)
    assert np.array_equal(ep, ep2) and np.array_equal(vp, vp2)


@pytest.mark.parametrize("levels", [1, 2, 5, 12])
def test_bitreverse_path_is_perfect_binary(levels):
    t = gen.path_bitrev(levels)
    n = t.n
    ep, vp = _run(t)
    j = np.arange(1, n, dtype=np.int64)               # edge k = j-1 sits between k and k+1
    tz = np.array([(int(x) & -int(x)).bit_length() - 1 for x in j])
    blk = 1 << (tz + 2)
    par = (j // blk) * blk + (1 << (tz + 1))
    want = np.where(par < n, par - 1, -1)
    assert np.array_equal(ep, want)
    # a vertex's parent is the odd one of its two edges (trailing-zero count 0)
    x = np.arange(n)
    jj = np.where(x % 2 == 1, x, x + 1)
    jj[n - 1] = n - 1
    assert np.array_equal(vp, jj - 1)
    assert invariants(n, t.u, t.v, t.w, ep, vp) == levels


# ---- dendrogram height (numerator of the paper's imbalance, Table 2) ----

@pytest.mark.parametrize("maker, want", [
    (lambda: gen.star(1000, 3), 999),           # one chain (Theorem lowerbound)
    (lambda: gen.path_mono(5000), 4999),        # one chain
    (lambda: gen.path_bitrev(10), 10),          # perfect binary: log2 n
    (lambda: gen.rrt(2, 0), 1),
])
def test_height_closed_forms(maker, want):
    t = maker()
    ep, vp = _run(t)
    assert oracle.dendrogram_height(ep, vp) == want


@pytest.mark.parametrize("seed", range(4))
def test_height_matches_independent_checker(seed):
    t = gen.shuffled(gen.rrt(4000, seed), seed) if seed % 2 else gen.caterpillar(4000, None, 1e-3, seed)
    ep, vp = _run(t)
    assert oracle.dendrogram_height(ep, vp) == invariants(t.n, t.u, t.v, t.w, ep, vp)


def test_height_degenerate_and_malformed():
    assert oracle.dendrogram_height(np.empty(0, np.int32), np.array([-1], np.int32)) == 0
    with pytest.raises(oracle.OracleError):      # a parent cycle
        oracle.dendrogram_height(np.array([1, 0], np.int32), np.array([0, 0, 1], np.int32))
    with pytest.raises(oracle.OracleError):      # a parent out of range
        oracle.dendrogram_height(np.array([5, -1], np.int32), np.array([0, 0, 1], np.int32))


# ---- library routine: scipy single linkage on the subdominant ultrametric ----

@pytest.mark.parametrize("seed", range(12))
def test_matches_scipy_single_linkage(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 120))
    t = gen.shuffled(gen.rrt(n, seed) if seed % 2 else gen.pref_attach(n, seed), seed)
    t.w[:] = rng.permutation(n - 1).astype(np.float32) * 0.5 + 1.0   # distinct weights
    ep, vp = _run(t)
    assert children_sets(n, ep, vp) == scipy_merges(n, t.u, t.v, t.w)


# ---- invariants (Section 3.1.2, Section 4.2, Theorem path_lcda, Corollary incident_ancestor) ----

@pytest.mark.parametrize("maker", [
    lambda: gen.rrt(3000, 3),
    lambda: gen.shuffled(gen.pref_attach(3000, 4), 4),
    lambda: gen.caterpillar(3000, None, 1e-3, 5),
    lambda: gen.shuffled(gen.caterpillar(2000, None, 1e-2, 6), 6),
    lambda: gen.rrt(3000, 7, weights="lognormal"),
])
def test_invariants_midsize(maker):
    t = maker()
    ep, vp = _run(t)
    invariants(t.n, t.u, t.v, t.w, ep, vp, lcda_pairs=30, seed=1)


# ---- error statuses ----

def test_error_statuses():
    u = np.array([1, 2], np.int32)
    v = np.array([0, 1], np.int32)
    w = np.array([0.1, 0.2], np.float32)
    assert oracle.dendrogram_status(3, u, v, w)[0] == oracle.OK
    assert oracle.dendrogram_status(0, u, v, w)[0] == oracle.INVALID_ARG
    assert oracle.dendrogram_status(3, np.array([1, 3], np.int32), v, w)[0] == oracle.BAD_VERTEX
    assert oracle.dendrogram_status(3, np.array([1, -1], np.int32), v, w)[0] == oracle.BAD_VERTEX
    assert oracle.dendrogram_status(3, u, v, np.array([0.1, np.nan], np.float32))[0] == oracle.NAN_WEIGHT
    # cycle (and therefore a disconnected vertex)
    assert oracle.dendrogram_status(3, np.array([1, 1], np.int32), np.array([0, 0], np.int32), w)[0] == oracle.NOT_A_TREE
    # self loop
    assert oracle.dendrogram_status(3, np.array([1, 2], np.int32), np.array([0, 2], np.int32), w)[0] == oracle.NOT_A_TREE


# ---- batched form: each tree is its own brute-force result ----

def test_batched_matches_per_tree_brute_force():
    trees = [gen.rrt(int(s), int(s)) for s in [1, 2, 5, 30, 1, 17]]
    trees.append(gen.shuffled(gen.caterpillar(25, None, 1e-1, 2), 2))
    f = gen.forest_from_trees(trees)
    ep, vp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
    for b, t in enumerate(trees):
        v0, v1 = int(f.voff[b]), int(f.voff[b + 1])
        e0, e1 = v0 - b, v1 - b - 1
        bep, bvp = brute_force(t.n, t.u, t.v, t.w)
        assert np.array_equal(ep[e0:e1], bep) and np.array_equal(vp[v0:v1], bvp)
