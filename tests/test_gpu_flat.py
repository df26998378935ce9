"""HDBSCAN* flat clusters on the GPU against the oracle, bit for bit: the
dendrogram, the labels and the stabilities.  Both sides take each
stability as the correctly rounded sum of the same fp64 terms (the oracle by
math.fsum, the GPU by exact fixed-point accumulation), so the excess-of-mass
decisions are the same too, near-ties included.  Edge cases: one and two
vertices, trees too small to split, invalid weights and sizes."""
import numpy as np
import pytest
import torch

import gen
import oracle
from oracle.flat_clusters import flat_clusters as oracle_flat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    pd.library()
    yield


def run(t, w, mcs):
    import paper_2401_06089_amd as pd
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    lab, st, ep, vp = pd.flat_clusters(d(t.u), d(t.v), d(w), mcs)
    return lab.cpu().numpy(), st.cpu().numpy(), ep.cpu().numpy(), vp.cpu().numpy()


def check(t, w, mcs):
    print(f"flat clusters n={t.n} mcs={mcs}", flush=True)
    lab, st, ep, vp = run(t, w, mcs)
    oep, ovp = oracle.dendrogram(t.n, t.u, t.v, w)
    assert np.array_equal(ep, oep) and np.array_equal(vp, ovp)
    olab, ost = oracle_flat(t.n, t.u, t.v, w, mcs)
    assert np.array_equal(lab, olab)
    assert st.dtype == ost.dtype and np.array_equal(st.view(np.uint64), ost.view(np.uint64))
    return olab, ost


def positive(w):
    return np.maximum(np.asarray(w, np.float32), np.float32(1e-7))


@pytest.mark.parametrize("maker", [
    lambda: gen.rrt(3_000, 1, weights="lognormal"),
    lambda: gen.rrt(40_000, 2, weights="lognormal"),
    lambda: gen.shuffled(gen.pref_attach(60_000, 3), 3),
    lambda: gen.caterpillar(50_000, None, 1e-3, 4),
    lambda: gen.shuffled(gen.rrt(150_000, 5, weights="lognormal"), 5),
    lambda: gen.star(5_001, 6),
], ids=["rrt3k", "rrt40k", "pa60k", "caterpillar", "rrt150k_shuf", "star"])
@pytest.mark.parametrize("mcs", [2, 7, 50])
def test_matches_oracle(maker, mcs):
    t = maker()
    olab, ost = check(t, positive(t.w), mcs)
    if t.n >= 40_000 and mcs <= 7:
        assert ost.size > 3          # the case exercises real selection work


def test_many_clusters_and_deep_cluster_tree():
    """Well-separated groups of rising sizes chained by heavier and heavier
    bridges: a deep cluster tree, many chosen clusters."""
    rng = np.random.default_rng(7)
    u, v, w = [], [], []
    start = 0
    prev_center = None
    for g in range(300):
        size = 20 + g % 13
        center = start
        for k in range(1, size):
            u.append(center)
            v.append(start + k)
            w.append(np.float32(rng.uniform(0.1, 0.2)))
        if prev_center is not None:
            u.append(prev_center)
            v.append(center)
            w.append(np.float32(1.0 + g))
        prev_center = center
        start += size
    t = gen.Tree(start, np.array(u, np.int32), np.array(v, np.int32), np.array(w, np.float32))
    for mcs in (5, 19):
        olab, ost = check(t, t.w, mcs)
        assert ost.size >= 250


def test_exact_ties_follow_the_tie_rule():
    """Dyadic weights: every stability is an exact small dyadic number on both
    sides, so exact ties (the parent wins) must come out the same."""
    rng = np.random.default_rng(11)
    for trial in range(30):
        t = gen.rrt(int(rng.integers(200, 3000)), int(rng.integers(1 << 30)))
        w = (2.0 ** rng.integers(-1, 2, t.n - 1)).astype(np.float32)
        lab, st, ep, vp = run(t, w, 3)
        olab, ost = oracle_flat(t.n, t.u, t.v, w, 3)
        assert np.array_equal(lab, olab) and np.array_equal(st, ost), trial


def test_near_ties_match_exactly():
    """Weights from {3, 6, 12}: their inverses are inexact in fp64, and many
    excess-of-mass comparisons are ties in real arithmetic, so they lie within
    the fp64 summation error bound of a tie, where a summation order other
    than the exact one could decide differently.  The labels and stabilities
    must still be the oracle's, bit for bit."""
    from oracle.flat_clusters import decisions_safe
    rng = np.random.default_rng(23)
    unsafe = 0
    for trial in range(40):
        t = gen.rrt(int(rng.integers(300, 4000)), int(rng.integers(1 << 30)))
        w = np.array([3.0, 6.0, 12.0], np.float32)[rng.integers(0, 3, t.n - 1)]
        mcs = int(rng.integers(2, 5))
        lab, st, ep, vp = run(t, w, mcs)
        olab, ost, info = oracle_flat(t.n, t.u, t.v, w, mcs, return_info=True)
        unsafe += not decisions_safe(info)
        assert np.array_equal(lab, olab), trial
        assert np.array_equal(st.view(np.uint64), ost.view(np.uint64)), trial
    assert unsafe > 0          # the set really holds near-ties


def test_degenerate_sizes_and_errors():
    import paper_2401_06089_amd as pd
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    e32 = np.empty(0, np.int32)
    lab, st, ep, vp = pd.flat_clusters(d(e32), d(e32), d(np.empty(0, np.float32)), 5)
    assert lab.cpu().tolist() == [-1] and vp.cpu().tolist() == [-1] and st.numel() == 0
    t = gen.rrt(2, 0)
    lab, st, _, _ = run(t, positive(t.w), 2)
    assert lab.tolist() == [-1, -1] and st.size == 0
    t = gen.rrt(30, 1)
    lab, st, _, _ = run(t, positive(t.w), 16)          # n < 2 * mcs: no split is possible
    assert (lab == -1).all() and st.size == 0
    t = gen.rrt(500, 2)
    for bad in (0.0, -1.0):
        w = positive(t.w)
        w[17] = bad
        with pytest.raises(pd.PandoraError) as ei:
            run(t, w, 5)
        assert ei.value.status == pd.INVALID_ARG
    with pytest.raises(pd.PandoraError) as ei:
        run(t, positive(t.w), 1)
    assert ei.value.status == pd.INVALID_ARG
    w = positive(t.w)
    w[3] = np.float32("nan")
    with pytest.raises(pd.PandoraError) as ei:
        run(t, w, 5)
    assert ei.value.status == pd.NAN_WEIGHT
    # the stream's workspace is fine afterwards
    check(gen.rrt(5000, 9, weights="lognormal"), positive(gen.rrt(5000, 9, weights="lognormal").w), 5)


def test_large_tree_sampled_properties():
    """2,000,000 vertices (several scan tiles per level, every level path):
    against the oracle."""
    t = gen.rrt(2_000_000, 12, weights="lognormal")
    check(t, positive(t.w), 20)


def test_full_size_c3_matches_oracle_hashes():
    """The benchmark's tree (preferential attachment, 50,000,000 vertices,
    mcs = 100), as bench.py runs it: labels and stabilities bit for bit the
    oracle's.  The oracle needs several minutes at this size, so its output
    enters as SHA-256 hashes written by tests/golden/make_golden.py (which
    calls only the generators and the oracle)."""
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hashes.json")) as f:
        g = json.load(f)["c3flat_pa_5e7_seed0_mcs100"]
    t = gen.c3_pref_attach(0)
    sha = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
    assert sha(np.concatenate([t.u.view(np.uint8), t.v.view(np.uint8), t.w.view(np.uint8)])) == g["input_sha256"]
    print(f"flat clusters n={t.n} mcs=100", flush=True)
    lab, st, ep, vp = run(t, t.w, g["min_cluster_size"])
    assert st.size == g["clusters"]
    assert sha(lab) == g["labels_sha256"]
    assert sha(st) == g["stability_sha256"]
    # and the properties any valid labelling has
    counts = np.bincount(lab[lab >= 0], minlength=st.size)
    assert (counts >= 100).all() and (st > 0).all()
