"""Stored fixtures: input drift guard and oracle regression (no GPU).
tests/golden/hashes.json is written by tests/golden/make_golden.py, which calls
only the generators and the oracle."""
import hashlib
import json
import os

import pytest

import gen
import oracle
from checks import invariants

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "hashes.json")) as f:
    GOLDEN = json.load(f)

MAKERS = {
    "c1_rrt_1e5_seed0": lambda: gen.c1_rrt(0),
    "rrt_1e6_seed0": lambda: gen.rrt(1_000_000, 0),
    "caterpillar_1e6_seed0": lambda: gen.c2b_caterpillar(0, n=1_000_000),
    "pref_attach_1e6_seed0": lambda: gen.c3_pref_attach(0, n=1_000_000),
}


def _sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(a.tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_generator_and_oracle_hashes(name):
    t = MAKERS[name]()
    g = GOLDEN[name]
    assert t.n == g["n"]
    assert _sha(t.u, t.v, t.w) == g["input_sha256"], "generator drift"
    ep, vp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    assert _sha(ep, vp) == g["oracle_output_sha256"], "oracle output changed"


def test_c1_invariants():
    t = gen.c1_rrt(0)
    ep, vp = oracle.dendrogram(t.n, t.u, t.v, t.w)
    invariants(t.n, t.u, t.v, t.w, ep, vp)
