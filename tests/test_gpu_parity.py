"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Inputs are seeded synthetic trees; sizes span one tile up to many tiles with
ragged tails, both sides of the LDS-tail thresholds (4096 edges, 8192
vertices), the adversarial shapes (monotone path: pointer depth n; star: one
chain; constant weights: all ties), and the full-size workloads.
"""
import itertools
import os

import numpy as np
import pytest
import torch

import gen
import oracle
from checks import prufer_trees
from gpu_util import assert_matches_oracle, gpu_dendrogram, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    pd.library()
    yield


SMALL = [
    ("n2", lambda: gen.rrt(2, 0)),
    ("n3", lambda: gen.rrt(3, 1)),
    ("rrt100", lambda: gen.rrt(100, 2)),
    ("rrt4097", lambda: gen.rrt(4097, 3)),        # m = 4096: tail takes level 0
    ("rrt4098", lambda: gen.rrt(4098, 4)),        # m = 4097: one global level
    ("rrt5000_shuf", lambda: gen.shuffled(gen.rrt(5000, 5), 5)),
    ("rrt70001", lambda: gen.rrt(70001, 6)),
    ("c1_rrt_1e5", lambda: gen.c1_rrt(0)),
    ("pa_3e5_shuf", lambda: gen.shuffled(gen.pref_attach(300_000, 7), 7)),
    ("caterpillar_2e5", lambda: gen.caterpillar(200_000, None, 1e-3, 8)),
    ("caterpillar_shuf", lambda: gen.shuffled(gen.caterpillar(123_457, None, 1e-2, 9), 9)),
    ("rrt_lognormal", lambda: gen.rrt(150_001, 10, weights="lognormal")),
]


@pytest.mark.parametrize("name,maker", SMALL, ids=[s[0] for s in SMALL])
def test_parity_shapes(name, maker):
    assert_matches_oracle(maker(), name)


@pytest.mark.parametrize("n", [2, 5, 4097, 4098, 100_000, 1_000_003])
def test_parity_monotone_path(n):
    """Pointer chains of depth n-1 at level 0 (many jump rounds)."""
    assert_matches_oracle(gen.path_mono(n), f"path{n}")
    t = gen.path_mono(n)
    t.w[:] = t.w[::-1].copy()                     # falling weights: root at the other end
    assert_matches_oracle(t, f"path_desc{n}")


@pytest.mark.parametrize("n", [3, 4097, 262_145])
def test_parity_star(n):
    assert_matches_oracle(gen.star(n, n), f"star{n}")


@pytest.mark.parametrize("levels", [3, 12, 17])
def test_parity_bitreverse_path(levels):
    assert_matches_oracle(gen.path_bitrev(levels), f"bitrev{levels}")


def test_parity_ties_and_signed_zero():
    t = gen.shuffled(gen.rrt(200_000, 11), 11)
    rng = np.random.default_rng(11)
    t.w[:] = rng.integers(0, 4, t.m).astype(np.float32)   # four distinct values only
    t.w[rng.random(t.m) < 0.3] = -0.0
    t.w[:50] = np.inf
    t.w[50:80] = -np.inf
    assert_matches_oracle(t, "ties")
    t.w[:] = 1.0                                          # every weight equal
    assert_matches_oracle(t, "constant")


def test_parity_exhaustive_tiny_forest():
    """All labelled trees on <= 5 vertices with every weight order and every 0/1
    weight pattern, as one batched forest; each tree checked against the oracle."""
    import paper_2401_06089_amd as pd
    trees = []
    for n in range(2, 6):
        for edges in prufer_trees(n):
            u = np.array([e[0] for e in edges], np.int32)
            v = np.array([e[1] for e in edges], np.int32)
            for p in itertools.permutations(range(n - 1)):
                trees.append(gen.Tree(n, u, v, np.array(p, np.float32)))
            for b in itertools.product([0, 1], repeat=n - 1):
                trees.append(gen.Tree(n, u, v, np.array(b, np.float32)))
    trees.append(gen.Tree(1, np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0, np.float32)))
    f = gen.forest_from_trees(trees)
    u, v, w = (torch.from_numpy(a).cuda() for a in (f.u, f.v, f.w))
    ep, vp = pd.dendrogram_batched(f.voff, u, v, w)
    oep, ovp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
    assert np.array_equal(vp.cpu().numpy(), ovp)
    assert np.array_equal(ep.cpu().numpy(), oep)


def test_single_vertex():
    import paper_2401_06089_amd as pd
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    ep, vp = pd.dendrogram(e, e, torch.empty(0, dtype=torch.float32, device="cuda"), n=1)
    assert ep.numel() == 0 and vp.cpu().tolist() == [-1]


def test_deterministic_repeat():
    t = gen.shuffled(gen.pref_attach(500_000, 12), 12)
    a = gpu_dendrogram(t)
    b = gpu_dendrogram(t)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_error_statuses():
    import paper_2401_06089_amd as pd
    base = gen.rrt(10_000, 13)

    def status(t):
        u, v, w = to_dev(t)
        ep = torch.empty(t.m, dtype=torch.int32, device="cuda")
        vp = torch.empty(t.n, dtype=torch.int32, device="cuda")
        st = pd.dendrogram_into(t.n, u, v, w, ep, vp)
        torch.cuda.synchronize()
        return st

    assert status(base) == pd.OK
    t = gen.Tree(base.n, base.u.copy(), base.v, base.w)
    t.u[777] = base.n                       # out of range
    assert status(t) == pd.BAD_VERTEX
    t.u[777] = -5
    assert status(t) == pd.BAD_VERTEX
    t = gen.Tree(base.n, base.u, base.v, base.w.copy())
    t.w[123] = np.nan
    assert status(t) == pd.NAN_WEIGHT
    t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w)
    t.u[500], t.v[500] = t.u[499], t.v[499]  # duplicate edge -> cycle + isolated vertex
    assert status(t) == pd.NOT_A_TREE
    t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w)
    t.v[42] = t.u[42]                        # self loop
    assert status(t) == pd.NOT_A_TREE
    big = gen.rrt(300_000, 14)
    t = gen.Tree(big.n, big.u.copy(), big.v.copy(), big.w)
    t.u[1000], t.v[1000] = t.u[2000], t.v[2000]
    assert status(t) == pd.NOT_A_TREE
    assert status(big) == pd.OK              # the library recovers after errors


@pytest.mark.parametrize("which", ["c2a_rrt_1e7", "c2b_caterpillar_1e7"])
def test_parity_full_size_1e7(which):
    t = gen.c2a_rrt(0) if which.startswith("c2a") else gen.c2b_caterpillar(0)
    assert_matches_oracle(t, which)


def test_parity_full_size_c3_5e7():
    t = gen.c3_pref_attach(0)
    assert_matches_oracle(t, "c3_pa_5e7")
