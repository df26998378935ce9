"""Autotuner: builds a table on small sizes, the table is applied per call,
and tuned calls still give the oracle's result bit for bit."""
import json

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_matches_oracle

pytestmark = pytest.mark.gpu


def test_autotune_table_and_tuned_parity(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    from paper_2401_06089_amd import autotune
    table = autotune.build_table([2_000, 60_000], seed=3, log=lambda *a: None)
    assert table["arch"].startswith("gfx")
    assert len(table["buckets"]) == 2 and table["buckets"][-1]["max_edges"] == 2**31 - 1
    path = tmp_path / "tune.json"
    path.write_text(json.dumps(table))
    autotune.install(autotune.load(str(path)))
    try:
        for t in (gen.rrt(2_000, 1), gen.shuffled(gen.caterpillar(60_000, None, 1e-3, 2), 2),
                  gen.path_mono(70_000)):
            assert_matches_oracle(t, "tuned")
        f = gen.forest_from_trees([gen.rrt(s, s) for s in (5, 3000, 1, 900)])
        u, v, w = (torch.from_numpy(a).cuda() for a in (f.u, f.v, f.w))
        ep, vp = pd.dendrogram_batched(f.voff, u, v, w)
        oep, ovp = oracle.dendrogram_batched(f.voff, f.u, f.v, f.w)
        assert np.array_equal(ep.cpu().numpy(), oep) and np.array_equal(vp.cpu().numpy(), ovp)
    finally:
        autotune.install(None)
        pd.set_thread_tuning(None)


def test_every_tile_config_matches_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06089_amd as pd
    from paper_2401_06089_amd import autotune
    autotune.install(None)            # no per-call table: the settings below apply
    t = gen.shuffled(gen.pref_attach(123_457, 5), 5)
    try:
        for cfg in range(4):
            for bits in (8, 9):
                pd.set_thread_tuning(dict(sync_free_max_edges=0, jump_steps=16, chain_digit_bits=bits,
                                          sort_tile_cfg=cfg))
                assert_matches_oracle(t, f"cfg{cfg}/bits{bits}")
    finally:
        pd.set_thread_tuning(None)
