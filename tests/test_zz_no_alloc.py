"""The entry point that allocates nothing (pandora_dendrogram_noalloc),
called through the C ABI: two calls in a row on the library's fixed scratch
array, the second with a smaller tree, each equal to pandora_dendrogram's
result on the same input and to the oracle, bit for bit; the size limit and
the one-vertex tree."""
import ctypes

import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    pd.library()
    return pd


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _call(pd, fn, t):
    u, v, w = _dev(t.u), _dev(t.v), _dev(t.w)
    ep = torch.full((t.m,), -7, dtype=torch.int32, device="cuda")
    vp = torch.full((t.n,), -7, dtype=torch.int32, device="cuda")
    st = fn(t.n, u, v, w, ep, vp)
    torch.cuda.synchronize()
    return st, ep.cpu().numpy(), vp.cpu().numpy()


def test_two_calls_match_plain_entry_and_oracle(pd):
    big = gen.shuffled(gen.pref_attach(pd.NOALLOC_MAX_VERTICES, 11), 11)
    small = gen.rrt(30_001, 12)
    for t in (big, small):
        print(f"noalloc n={t.n}", flush=True)
        st, ep, vp = _call(pd, pd.dendrogram_noalloc_into, t)
        assert st == pd.OK, pd.status_string(st)
        st2, ep2, vp2 = _call(pd, pd.dendrogram_into, t)
        assert st2 == pd.OK
        assert np.array_equal(ep, ep2) and np.array_equal(vp, vp2)
        oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
        assert np.array_equal(ep, oep) and np.array_equal(vp, ovp)


def test_limits_and_degenerate_sizes(pd):
    lib = pd.library()
    assert lib.pandora_workspace_bytes(pd.NOALLOC_MAX_VERTICES, 1) <= pd.NOALLOC_SCRATCH_BYTES
    assert lib.pandora_workspace_bytes(pd.NOALLOC_MAX_VERTICES + 1, 1) > pd.NOALLOC_SCRATCH_BYTES
    t = gen.rrt(pd.NOALLOC_MAX_VERTICES + 1, 13)
    st, ep, vp = _call(pd, pd.dendrogram_noalloc_into, t)
    assert st == pd.OUT_OF_MEMORY
    assert (ep == -7).all() and (vp == -7).all()        # rejected before any work
    one = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    assert pd.dendrogram_noalloc_into(1, None, None, None, None, one) == pd.OK
    torch.cuda.synchronize()
    assert int(one.item()) == -1
    two = gen.rrt(2, 14)
    st, ep, vp = _call(pd, pd.dendrogram_noalloc_into, two)
    assert st == pd.OK and ep.tolist() == [-1] and vp.tolist() == [0, 0]
    assert lib.pandora_dendrogram_noalloc(0, None, None, None, None, None, None) == pd.INVALID_ARG


def test_input_error_then_recovery(pd):
    t = gen.rrt(5_000, 15)
    bad = gen.Tree(t.n, t.u.copy(), t.v.copy(), t.w.copy())
    bad.w[17] = np.float32("nan")
    st, _, _ = _call(pd, pd.dendrogram_noalloc_into, bad)
    assert st == pd.NAN_WEIGHT
    st, ep, vp = _call(pd, pd.dendrogram_noalloc_into, t)
    assert st == pd.OK
    oep, ovp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    assert np.array_equal(ep, oep) and np.array_equal(vp, ovp)
