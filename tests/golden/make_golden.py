"""Writes tests/golden/hashes.json: SHA-256 of seeded generator outputs (drift
guard for the inputs) and of the oracle's outputs on them.  Calls only the
generators and the oracle; nothing here comes from the GPU path.

    python tests/golden/make_golden.py            # the dendrogram cases
    python tests/golden/make_golden.py --c3flat   # also the full-size flat clusters (slow)

The flat-cluster entry holds the oracle's HDBSCAN* labels and stabilities
for the 50,000,000-vertex preferential-attachment tree at minimum cluster
size 100 (the benchmark's flat-cluster workload); the oracle takes several
minutes there, so the GPU test compares against these hashes.
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


FLAT_CASES = {
    "c3flat_pa_5e7_seed0_mcs100": (lambda: gen.c3_pref_attach(0), 100),
}


def main():
    path = os.path.join(HERE, "hashes.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    if "--c3flat" in sys.argv:
        from oracle.flat_clusters import flat_clusters
        for name, (make, mcs) in FLAT_CASES.items():
            t = make()
            lab, st = flat_clusters(t.n, t.u, t.v, t.w, mcs)
            out[name] = {"n": t.n, "min_cluster_size": mcs, "input_sha256": sha(t.u, t.v, t.w),
                         "clusters": int(st.size), "labels_sha256": sha(lab),
                         "stability_sha256": sha(st), "stability_sum": float(st.sum())}
    for name, make in CASES.items():
        t = make()
        ep, vp = oracle.dendrogram(t.n, t.u, t.v, t.w)
        out[name] = {"n": t.n, "input_sha256": sha(t.u, t.v, t.w),
                     "oracle_output_sha256": sha(ep, vp)}
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
