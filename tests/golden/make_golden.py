"""Writes tests/golden/hashes.json: SHA-256 of seeded generator outputs (drift
guard for the inputs) and of the oracle's outputs on them.  Calls only the
generators and the oracle; nothing here comes from the GPU path.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen      # noqa: E402
import oracle   # noqa: E402


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(a.tobytes())
    return h.hexdigest()


CASES = {
    "c1_rrt_1e5_seed0": lambda: gen.c1_rrt(0),
    "rrt_1e6_seed0": lambda: gen.rrt(1_000_000, 0),
    "caterpillar_1e6_seed0": lambda: gen.c2b_caterpillar(0, n=1_000_000),
    "pref_attach_1e6_seed0": lambda: gen.c3_pref_attach(0, n=1_000_000),
}


def main():
    out = {}
    for name, make in CASES.items():
        t = make()
        ep, vp = oracle.dendrogram(t.n, t.u, t.v, t.w)
        out[name] = {"n": t.n, "input_sha256": sha(t.u, t.v, t.w),
                     "oracle_output_sha256": sha(ep, vp)}
    with open(os.path.join(HERE, "hashes.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
