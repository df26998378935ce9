"""The multithreaded CPU form of the path gives the oracle's result bit for
bit: every small labelled tree with every weight order and tie pattern, the
benchmark shapes, ties and signed zeros, any thread count, and the error
statuses of the GPU library."""
import itertools
import os

import numpy as np
import pytest

import gen
import oracle
from checks import prufer_trees


@pytest.fixture(scope="module")
def cpu():
    from paper_2401_06089_amd import cpu as c
    if not os.path.exists(c.LIB_PATH):
        c.build()
    return c


def same(cpu, t, threads=0):
    ep, vp = cpu.dendrogram(t.n, t.u, t.v, t.w, threads=threads)
    oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    return np.array_equal(ep, oep) and np.array_equal(vp, ovp)


def test_every_small_tree(cpu):
    """Every labelled tree on n <= 5 vertices with every weight order and every
    0/1 pattern; n = 6 with sampled weights."""
    rng = np.random.default_rng(3)
    count = 0
    for n in range(2, 7):
        for edges in prufer_trees(n):
            u = np.array([e[0] for e in edges], np.int32)
            v = np.array([e[1] for e in edges], np.int32)
            if n <= 5:
                weights = [np.array(p, np.float32) for p in itertools.permutations(range(n - 1))]
                weights += [np.array(b, np.float32) for b in itertools.product([0, 1], repeat=n - 1)]
            else:
                weights = [rng.permutation(n - 1).astype(np.float32), rng.integers(0, 2, n - 1).astype(np.float32)]
            for w in weights:
                ep, vp = cpu.dendrogram(n, u, v, w, threads=2)
                oep, ovp = oracle.dendrogram(n, u, v, w)
                assert np.array_equal(ep, oep) and np.array_equal(vp, ovp), (edges, w)
                count += 1
    assert count > 7500


@pytest.mark.parametrize("maker", [
    lambda: gen.rrt(2, 0),
    lambda: gen.rrt(30_000, 1),
    lambda: gen.shuffled(gen.rrt(50_000, 2), 2),
    lambda: gen.caterpillar(120_000, None, 1e-3, 3),
    lambda: gen.shuffled(gen.pref_attach(150_000, 4), 4),
    lambda: gen.star(40_001, 5),
    lambda: gen.path_mono(100_000),
    lambda: gen.path_bitrev(14),
    lambda: gen.c1_rrt(0),
], ids=["n2", "rrt", "rrt_shuf", "caterpillar", "pa_shuf", "star", "path_mono", "bitrev", "c1"])
def test_shapes(cpu, maker):
    assert same(cpu, maker())


def test_ties_signed_zero_and_infinities(cpu):
    t = gen.shuffled(gen.rrt(20_000, 6), 6)
    w = t.w.copy()
    w[::3] = 0.5
    w[1::7] = -0.0
    w[2::7] = 0.0
    w[5::11] = np.float32("inf")
    w[6::13] = np.float32("-inf")
    t = gen.Tree(t.n, t.u, t.v, w)
    assert same(cpu, t)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_any_thread_count(cpu, threads):
    assert same(cpu, gen.shuffled(gen.pref_attach(60_000, 7), 7), threads=threads)


def test_single_vertex(cpu):
    ep, vp = cpu.dendrogram(1, np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float32))
    assert ep.size == 0 and list(vp) == [-1]


def test_error_statuses(cpu):
    base = gen.rrt(5000, 8)
    cases = {}
    t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w.copy())
    t.v[10] = base.n + 1
    cases["bad"] = (t, 6)
    t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w.copy())
    t.w[3] = np.float32("nan")
    cases["nan"] = (t, 3)
    t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w.copy())
    t.u[40], t.v[40] = t.u[90], t.v[90]                 # a repeated edge: cycle + disconnected
    cases["cycle"] = (t, 2)
    t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w.copy())
    t.v[42] = t.u[42]
    cases["selfloop"] = (t, 2)
    for name, (t, want) in cases.items():
        st, _, _ = cpu.dendrogram_status(t.n, t.u, t.v, t.w)
        ost, _, _ = oracle.dendrogram_status(t.n, t.u, t.v, t.w)
        assert st == want == ost, name
    st, _, _ = cpu.dendrogram_status(0, np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float32))
    assert st == 1
