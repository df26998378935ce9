"""Autotuner for libpandora's speed knobs.

Knobs (``pandora_tuning_t``): the radix tile (1024 to 8192 keys per
workgroup), pointer-jumping steps per launch, the chain sort's digit width,
and whether the level loop runs without host round trips.  None of them
changes a result; they trade launch count, parallelism and scatter
contiguity, and the best choice depends on the input size.

For each size bucket the tuner builds trees on the device (random recursive
trees with uniform weights and noisy rising paths, from torch's seeded RNG),
then sweeps one knob at a time (coordinate descent, two rounds) timing the
median of several calls, and keeps the fastest setting.  The table is written
as JSON keyed by the GPU architecture; ``install`` makes the binding apply the
matching entry to every call from then on (as a per-thread override).

    python -m paper_2401_06089_amd.autotune --out tuning_gfx950.json
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import time
from typing import Dict, List, Optional

import torch

from . import Tuning, _load, dendrogram_into, get_tuning, set_thread_tuning  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))

KNOBS = {
    "sort_tile_cfg": [0, 1, 2, 3],
    "jump_steps": [4, 8, 16, 32],
    "chain_digit_bits": [8, 9],
    "sync_free_max_edges": [0, 2**31 - 1],
    "persist_max_edges": [0, 1 << 16, 1 << 18],
}

DEFAULT_SIZES = [1_000, 10_000, 100_000, 1_000_000, 10_000_000]


def arch_name() -> str:
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def _device_trees(n: int, seed: int, device) -> list:
    """Two input shapes of n vertices, built on the device."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    i = torch.arange(1, n, device=device, dtype=torch.float64)
    parent = torch.floor(torch.rand(n - 1, generator=g, device=device, dtype=torch.float64) * i)
    u = torch.arange(1, n, device=device, dtype=torch.int32)
    v = parent.to(torch.int32)
    w = torch.rand(n - 1, generator=g, device=device, dtype=torch.float32)
    # a path whose weights rise with small noise: deep contraction pointers
    pu = torch.arange(0, n - 1, device=device, dtype=torch.int32)
    pv = pu + 1
    pw = (torch.arange(0, n - 1, device=device, dtype=torch.float32) / max(n - 1, 1)
          + 1e-3 * torch.rand(n - 1, generator=g, device=device, dtype=torch.float32))
    return [(n, u, v, w), (n, pu, pv, pw)]


def _time_setting(trees, tuning: dict, reps: int) -> float:
    # an installed table would replace the candidate on every call: suspend it
    import paper_2401_06089_amd as pkg
    hook = pkg._tuning_hook
    pkg._set_tuning_hook(None)
    set_thread_tuning(tuning)
    try:
        outs = [(torch.empty(t[0] - 1, dtype=torch.int32, device=t[1].device),
                 torch.empty(t[0], dtype=torch.int32, device=t[1].device)) for t in trees]
        for (n, u, v, w), (ep, vp) in zip(trees, outs):     # warm-up (scratch growth)
            st = dendrogram_into(n, u, v, w, ep, vp)
            if st != 0:
                raise RuntimeError(f"status {st} while tuning")
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            for (n, u, v, w), (ep, vp) in zip(trees, outs):
                dendrogram_into(n, u, v, w, ep, vp)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - a)
        return statistics.median(times) * 1e3
    finally:
        set_thread_tuning(None)
        pkg._set_tuning_hook(hook)


def tune_size(n: int, seed: int = 0, rounds: int = 2, reps: Optional[int] = None, log=print) -> dict:
    device = torch.device("cuda:0")
    trees = _device_trees(n, seed, device)
    if reps is None:
        reps = 21 if n <= 100_000 else (9 if n <= 2_000_000 else 5)
    best = dict(get_tuning())
    best_ms = _time_setting(trees, best, reps)
    for _ in range(rounds):
        changed = False
        for knob, values in KNOBS.items():
            for val in values:
                if best[knob] == val:
                    continue
                cand = dict(best, **{knob: val})
                ms = _time_setting(trees, cand, reps)
                if ms < best_ms * 0.98:          # require a clear win
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    log(f"n={n}: {best_ms:.3f} ms per pair of trees with {best}")
    return {"n": n, "tuning": best, "ms": best_ms}


def build_table(sizes: List[int] = DEFAULT_SIZES, seed: int = 0, log=print) -> dict:
    # an installed table would override every candidate: tune without one
    install(None)
    results = [tune_size(n, seed, log=log) for n in sizes]
    buckets = []
    for k, r in enumerate(results):
        # bucket boundary: geometric midpoint to the next tuned size (edges)
        hi = int((sizes[k] * sizes[k + 1]) ** 0.5) if k + 1 < len(sizes) else 2**31 - 1
        buckets.append({"max_edges": hi, "tuning": r["tuning"], "tuned_n": r["n"], "ms": r["ms"]})
    return {"arch": arch_name(), "buckets": buckets}


_table: Optional[List[dict]] = None


def install(table: Optional[dict]) -> None:
    """Apply `table` (from build_table / a JSON file) to every later call; None removes it."""
    global _table
    from . import _set_tuning_hook
    if table is None:
        _table = None
        _set_tuning_hook(None)
        return
    # knobs a table does not name keep the process-wide values
    base = get_tuning()
    _table = sorted(({**b, "tuning": {**base, **b["tuning"]}} for b in table["buckets"]),
                    key=lambda b: b["max_edges"])
    _set_tuning_hook(pick)


def pick(edges: int) -> Optional[dict]:
    if not _table:
        return None
    for b in _table:
        if edges <= b["max_edges"]:
            return b["tuning"]
    return _table[-1]["tuning"]


def load(path: Optional[str] = None) -> Optional[dict]:
    """Read a tuning table: `path`, else $PANDORA_TUNE_CACHE, else the table
    shipped for this GPU architecture (tuning_<arch>.json next to this file)."""
    cands = [path, os.environ.get("PANDORA_TUNE_CACHE")]
    if torch.cuda.is_available():
        cands.append(os.path.join(_HERE, f"tuning_{arch_name()}.json"))
    for c in cands:
        if c and os.path.exists(c):
            with open(c) as f:
                t = json.load(f)
            if torch.cuda.is_available() and t.get("arch") not in (None, arch_name()):
                continue
            return t
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="JSON path (default: tuning_<arch>.json in the package)")
    ap.add_argument("--sizes", default=",".join(str(s) for s in DEFAULT_SIZES))
    args = ap.parse_args()
    _load()
    sizes = [int(x) for x in args.sizes.split(",")]
    table = build_table(sizes)
    out = args.out or os.path.join(_HERE, f"tuning_{table['arch']}.json")
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(out)


if __name__ == "__main__":
    main()
