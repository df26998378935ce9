"""The two level-loop modes (host-synchronised and sync-free) and the tuning
knobs change speed only: every mode gives the oracle's result bit for bit."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_matches_oracle

pytestmark = pytest.mark.gpu

MODES = {
    "synced": dict(sync_free_max_edges=0, jump_steps=16, chain_digit_bits=0, persist_max_edges=0),
    "syncfree": dict(sync_free_max_edges=2**31 - 1, jump_steps=16, chain_digit_bits=0, persist_max_edges=0),
    "syncfree_short_jumps_9bit": dict(sync_free_max_edges=2**31 - 1, jump_steps=2, chain_digit_bits=9,
                                      persist_max_edges=0),
    "synced_9bit": dict(sync_free_max_edges=0, jump_steps=4, chain_digit_bits=9, persist_max_edges=0),
    # every level in the persistent kernel, level 0 included
    "synced_persist_all": dict(sync_free_max_edges=0, jump_steps=16, chain_digit_bits=0,
                               persist_max_edges=2**31 - 1),
    "syncfree_persist_short_jumps": dict(sync_free_max_edges=2**31 - 1, jump_steps=1, chain_digit_bits=0,
                                         persist_max_edges=2**31 - 1),
    "synced_persist_mid": dict(sync_free_max_edges=0, jump_steps=16, chain_digit_bits=0,
                               persist_max_edges=1 << 15),
}


@pytest.fixture(params=sorted(MODES), autouse=True)
def mode(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    old = pd.set_tuning(**MODES[request.param])
    yield request.param
    pd.set_tuning(**old)


@pytest.mark.parametrize("maker", [
    lambda: gen.rrt(4098, 1),
    lambda: gen.shuffled(gen.rrt(70_001, 2), 2),
    lambda: gen.caterpillar(300_000, None, 1e-3, 3),
    lambda: gen.shuffled(gen.pref_attach(200_000, 4), 4),
    lambda: gen.path_mono(200_000),
    lambda: gen.star(50_001, 5),
    lambda: gen.path_bitrev(15),
], ids=["rrt4098", "rrt70k_shuf", "caterpillar300k", "pa200k_shuf", "path200k", "star50k", "bitrev15"])
def test_modes_parity(maker, mode):
    t = maker()
    assert_matches_oracle(t, mode)
    import paper_2401_06089_amd as pd
    st = pd.last_stats()
    assert st["sync_free"] == (1 if "syncfree" in mode else 0)
    if "persist_all" in mode or "persist_short" in mode:
        assert st["persistent"] == 1          # every tree here is larger than the LDS tail
    if "persist" not in mode:
        assert st["persistent"] == 0


def test_modes_forest(mode):
    import paper_2401_06089_amd as pd
    trees = [gen.rrt(int(n), s) for s, n in enumerate([1, 5, 9000, 3, 120_000, 2, 40_000])]
    trees += [gen.path_mono(3) for _ in range(9000)]
    f = gen.forest_from_trees(trees)
    u, v, w = (torch.from_numpy(a).cuda() for a in (f.u, f.v, f.w))
    ep, vp = pd.dendrogram_batched(f.voff, u, v, w)
    oep, ovp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
    assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)


def test_modes_errors(mode):
    import paper_2401_06089_amd as pd
    base = gen.rrt(50_000, 9)
    for kind in ("cycle", "selfloop", "bad"):
        t = gen.Tree(base.n, base.u.copy(), base.v.copy(), base.w)
        if kind == "cycle":
            t.u[700], t.v[700] = t.u[800], t.v[800]
        elif kind == "selfloop":
            t.v[42] = t.u[42]
        else:
            t.v[5] = base.n + 3
        u, v, w = (torch.from_numpy(a).cuda() for a in (t.u, t.v, t.w))
        ep = torch.empty(t.m, dtype=torch.int32, device="cuda")
        vp = torch.empty(t.n, dtype=torch.int32, device="cuda")
        st = pd.dendrogram_into(t.n, u, v, w, ep, vp)
        assert st == (pd.BAD_VERTEX if kind == "bad" else pd.NOT_A_TREE), (kind, st)
    assert_matches_oracle(base, mode)
