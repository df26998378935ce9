#!/usr/bin/env python3
"""Benchmark: single-linkage dendrograms of MSTs on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c3]

A step is one pass of the whole method (weight sort, contraction levels,
expansion, chain sort, stitch) over one batch of synthetic input that is
already resident in HBM.  The default workload is the largest single tree:
a preferential-attachment tree of 50,000,000 vertices with lognormal fp32
weights and 5 % ten-fold bridges, one call per step.

Printed: one JSON line with the throughput (MST edges per second), the
roofline of the dominant kernel (algorithmic bytes per launch over its mean
HIP-event duration on the library's stream, against 8 TB/s), the CPU oracle
timed on this host on the same inputs (its comparison sort on every host
thread and on one, each timed apart from the sequential union-find sweep),
and, for the default workload, two short side measurements: the 4,096-tree
forest in one batched call against one call per tree, and a short serving
run.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import statistics
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FLAT_MCS = 100   # minimum cluster size of the flat-cluster workloads
HDB_DIM, HDB_MIN_PTS = 3, 2

WORKLOADS = {
    "c2": "two single trees, n=10,000,000 each: (a) random recursive tree, fp32 uniform [0,1) "
          "weights; (b) caterpillar, 9,000,000-vertex spine + 1,000,000 leaves, spine weights "
          "rising along the path + fp32 uniform noise 1e-3; one call per tree",
    "c1": "random recursive tree, n=100,000, fp32 uniform weights",
    "c2a": "random recursive tree, n=10,000,000, fp32 uniform weights",
    "c2b": "caterpillar, n=10,000,000 (9,000,000 spine + 1,000,000 leaves)",
    "c3": "preferential-attachment tree, n=50,000,000, lognormal(0,1.5) fp32 weights, 5% x10 bridges",
    "c3flat": "HDBSCAN* flat clusters (min cluster size 100) of the preferential-attachment tree, "
              "n=50,000,000, lognormal(0,1.5) fp32 weights, 5% x10 bridges: dendrogram + clusters per call",
    "hdb3d": "HDBSCAN* end to end on uniform points in the unit cube (3D; 10,000,000 by default), min_pts 2, "
             "min cluster size 100: mutual-reachability MST (uniform grid), dendrogram and flat clusters per call",
    "c4": "4,096 trees, lognormal sizes in [100, 1,000,000] (~50M edges), half random-recursive "
          "half caterpillar, fp32 uniform weights, one batched call",
    "c5": "serving: Poisson arrivals at 2,000 req/s of random recursive trees with log-uniform "
          "sizes in [1,000, 10,000,000] and lognormal(0,1.5) fp32 weights, drawn from a "
          "device-resident pool, admitted by HBM footprint against a 200 GB budget",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(name):
    import gen
    if name == "c2":
        return [("tree", gen.c2a_rrt(0)), ("tree", gen.c2b_caterpillar(0))]
    if name == "c1":
        return [("tree", gen.c1_rrt(0))]
    if name == "c2a":
        return [("tree", gen.c2a_rrt(0))]
    if name == "c2b":
        return [("tree", gen.c2b_caterpillar(0))]
    if name == "c3":
        return [("tree", gen.c3_pref_attach(0))]
    if name == "c4":
        return [("forest", gen.c4_batched(0))]
    if name == "c3flat":
        return [("flat", gen.c3_pref_attach(0))]
    raise SystemExit(f"unknown workload {name}")


def committed_profile(workload):
    """The machine-readable part of the committed rocprofv3 counter summary
    for this workload (and its file), or (None, None) when there is none or
    the kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2401_06089_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    for md in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(md) as fh:
            text = fh.read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        if not m:
            continue
        try:
            data = json.loads(m.group(1))
        except ValueError:
            continue
        if data.get("workload") != workload or data.get("source_sha256") != h.hexdigest():
            continue
        return data, os.path.relpath(md, ROOT)
    return None, None


def committed_traffic(workload, kernel):
    """HBM bytes per dispatch of `kernel` from the committed counter summary."""
    data, md = committed_profile(workload)
    k = data.get("kernels", {}).get(kernel) if data else None
    if not k:
        return None
    return {"bytes_per_launch": k["traffic_bytes_per_dispatch"], "summary": md,
            "rocprof_avg_us": k["avg_us_rocprof"]}


def copy_bandwidth(dev) -> float:
    """Device-to-device copy of 1 GiB on this GPU, read plus write bytes per second (GB/s)."""
    import torch
    n = 1 << 28
    a = torch.empty(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbps = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def random_gather_rate(dev) -> dict:
    """The rate of independent random 4-byte gathers from a 1 GiB table on this
    GPU (torch.take of 2^26 uniform indices): the ceiling of kernels bound by
    random accesses, each of which moves a whole cache line."""
    import torch
    table = torch.zeros(1 << 28, dtype=torch.int32, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    idx = torch.randint(0, table.numel(), (1 << 26,), device=dev, generator=g)
    torch.take(table, idx)
    torch.cuda.synchronize()
    reps = 3
    a = time.perf_counter()
    for _ in range(reps):
        torch.take(table, idx)
    torch.cuda.synchronize()
    s = (time.perf_counter() - a) / reps
    del table, idx
    torch.cuda.empty_cache()
    return {"gathers_per_s": (1 << 26) / s, "table_bytes": 1 << 30}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-extras", action="store_true",
                    help="c3: skip the side measurements (batched forest, short serving run)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="capture each call once into a HIP graph and replay it every step")
    ap.add_argument("--compare-per-tree", action="store_true",
                    help="c4: also time the same trees built one call per tree")
    ap.add_argument("--duration", type=float, default=60.0, help="c5: seconds of arrivals")
    ap.add_argument("--discard", type=float, default=5.0, help="c5: warm-up seconds not reported")
    ap.add_argument("--rate", type=float, default=2000.0, help="c5: arrivals per second")
    ap.add_argument("--pool", type=int, default=512, help="c5: distinct trees in the device pool")
    ap.add_argument("--streams", type=int, default=2, help="c5: server slots (one stream each)")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="c5: admission budget")
    ap.add_argument("--max-batch-edges", type=int, default=8_000_000, help="c5: edge cap of one batch")
    ap.add_argument("--policy", default="small_first", choices=["fifo", "small_first"], help="c5: batching order")
    ap.add_argument("--points", type=int, default=10_000_000, help="hdb3d: points in the cloud")
    ap.add_argument("--sample-every", type=int, default=4,
                    help="bracket the dominant kernel with HIP events on every k-th timed step")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run two kernels of known traffic for scaling hardware byte counters: a "
                         "plain 1 GiB device-to-device copy, and 2^26 random 4-byte gathers from a 1 GiB "
                         "table (each must move at least one cache line)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py builds dendrograms on one GPU only; a tree or forest is not split across "
              "GPUs in this build (see DESIGN.md on sharding). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2401_06089_amd as pd

    pd.library()   # fails loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calibrate_copy:
        src = torch.ones(256 * 1024 * 1024, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del dst
        g = torch.Generator(device=dev)
        g.manual_seed(0)
        idx = torch.randint(0, src.numel(), (1 << 26,), device=dev, generator=g)
        torch.take(src, idx)
        torch.cuda.synchronize()
        del src, idx
        torch.cuda.empty_cache()

    if args.workload == "c5":
        return run_serving(args, dev)
    if args.workload == "hdb3d":
        return run_points(args, dev)

    t0 = time.time()
    items = make_inputs(args.workload)
    log(f"generated {args.workload} in {time.time() - t0:.1f}s")
    calls = []
    total_edges = 0
    total_vertices = 0
    for kind, obj in items:
        u = torch.from_numpy(obj.u).to(dev)
        v = torch.from_numpy(obj.v).to(dev)
        w = torch.from_numpy(obj.w).to(dev)
        if kind == "tree":
            ep = torch.empty(obj.m, dtype=torch.int32, device=dev)
            vp = torch.empty(obj.n, dtype=torch.int32, device=dev)
            calls.append(("tree", obj.n, u, v, w, ep, vp))
            total_edges += obj.m
            total_vertices += obj.n
        elif kind == "flat":
            ep = torch.empty(obj.m, dtype=torch.int32, device=dev)
            vp = torch.empty(obj.n, dtype=torch.int32, device=dev)
            lab = torch.empty(obj.n, dtype=torch.int32, device=dev)
            stab = torch.empty(obj.n // FLAT_MCS, dtype=torch.float64, device=dev)
            calls.append(("flat", obj.n, u, v, w, ep, vp, lab, stab))
            total_edges += obj.m
            total_vertices += obj.n
        else:
            calls.append(("forest", obj.voff, u, v, w))
            total_edges += obj.m_total
            total_vertices += obj.n_total
    torch.cuda.synchronize()

    if args.graph and any(c[0] == "flat" for c in calls):
        raise SystemExit("flat clusters read level sizes back during the call: no graph capture")
    graphs = []
    if args.graph:
        for c in calls:
            if c[0] == "tree":
                graphs.append(pd.Graph(c[2], c[3], c[4], n=c[1]))
            else:
                graphs.append(pd.Graph(c[2], c[3], c[4], voff=c[1]))

    flat_k = []

    def eager_step():
        for c in calls:
            if c[0] == "tree":
                st = pd.dendrogram_into(*c[1:])
                if st != pd.OK:
                    raise RuntimeError(f"status {st}: {pd.status_string(st)}")
            elif c[0] == "flat":
                n_, u_, v_, w_, ep_, vp_, lab_, stab_ = c[1:]
                st, k = pd.flat_clusters_into(n_, u_, v_, w_, FLAT_MCS, ep_, vp_, lab_, stab_)
                if st != pd.OK:
                    raise RuntimeError(f"status {st}: {pd.status_string(st)}")
                flat_k.append(k)
            else:
                pd.dendrogram_batched(c[1], c[2], c[3], c[4])

    def graph_step():
        for g in graphs:
            g.launch()

    step = graph_step if graphs else eager_step
    # Graph replays carry no per-kernel events: with --graph the kernel
    # breakdown and the dominant kernel's timing come from eager calls on the
    # same inputs, right after the timed replays.
    prof_step = eager_step

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # One profiled step (every kernel kind timed) picks the dominant kernel.
    pd.profile_enable(pd.PROFILE_ALL)
    prof_step()
    torch.cuda.synchronize()
    stages = pd.profile_read()
    dominant = max(stages, key=lambda k: stages[k]["ms"])
    dom_kind = stages[dominant]["kind"]

    # Timed region: the dominant kernel is bracketed with HIP events on every
    # args.sample_every-th step (a pair of events per launch costs a few
    # microseconds, which matters for small trees with many launches).
    lat = []
    dom = {"ms": 0.0, "bytes": 0.0, "launches": 0}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        sample = not graphs and i % args.sample_every == 0
        pd.profile_enable((1 << dom_kind) if sample else 0)
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        if sample:
            d = pd.profile_read()[dominant]
            for k in dom:
                dom[k] += d[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    if graphs:
        pd.profile_enable(1 << dom_kind)
        for _ in range(args.steps):
            prof_step()
        torch.cuda.synchronize()
        dom = pd.profile_read()[dominant]
    pd.profile_enable(0)

    ms_per_step = 1000.0 * elapsed / args.steps
    value = total_edges * args.steps / elapsed
    avg_launch_s = dom["ms"] / 1000.0 / max(dom["launches"], 1)
    bytes_per_launch = dom["bytes"] / max(dom["launches"], 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0

    out = {
        "metric": "MST edges/sec -> dendrogram",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "edges_per_step": total_edges, "vertices_per_step": total_vertices,
                   "calls_per_step": len(calls), "parallelism": "single GPU",
                   "hip_graph": bool(args.graph), "tuning": pd.get_tuning()},
        "mpoints_per_s": total_vertices * args.steps / elapsed / 1e6,
        "last_call_stats": pd.last_stats(),
        "latency_ms": {"p50": 1000 * statistics.median(lat),
                       "p99": 1000 * float(np.percentile(lat, 99)),
                       "per": "step"},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_launch_s * 1000,
                     "launches": dom["launches"],
                     "measured_on": ("eager calls after the timed graph replays" if graphs
                                     else f"every {args.sample_every}th timed step")},
        "path_hbm": {"algorithmic_bytes_per_step": sum(s["bytes"] for s in stages.values()),
                     "algorithmic_GBps": sum(s["bytes"] for s in stages.values()) / (ms_per_step / 1000) / 1e9},
    }
    out["path_hbm"]["frac"] = out["path_hbm"]["algorithmic_GBps"] / HBM_PEAK_GBS
    # The whole path's counter-measured HBM bytes per step (all library
    # kernels, from the committed rocprofv3 summary) over this run's step time.
    prof, prof_md = committed_profile(args.workload)
    if prof and prof.get("path") and not graphs:
        per_step = prof["path"]["traffic_bytes"] / prof["path"]["steps"]
        out["path_hbm"]["traffic_bytes_per_step"] = per_step
        out["path_hbm"]["traffic_GBps"] = per_step / (ms_per_step / 1000) / 1e9
        out["path_hbm"]["traffic_frac"] = out["path_hbm"]["traffic_GBps"] / HBM_PEAK_GBS
        out["path_hbm"]["traffic_source"] = prof_md
    out["roofline"]["copy_GBps"] = copy_bandwidth(dev)
    rg = random_gather_rate(dev)
    if prof and prof.get("calibration", {}).get("gather_bytes_per_access"):
        rg["line_bytes"] = prof["calibration"]["gather_bytes_per_access"]
        rg["line_GBps"] = rg["gathers_per_s"] * rg["line_bytes"] / 1e9
    out["roofline"]["random_gather"] = rg
    tr = committed_traffic(args.workload, dominant)
    if tr:
        out["roofline"]["traffic"] = tr["bytes_per_launch"]
        out["roofline"]["traffic_GBps"] = tr["bytes_per_launch"] / avg_launch_s / 1e9
        out["roofline"]["traffic_frac"] = out["roofline"]["traffic_GBps"] / HBM_PEAK_GBS
        out["roofline"]["traffic_source"] = tr["summary"]
        out["roofline"]["rocprof_avg_launch_ms"] = tr["rocprof_avg_us"] / 1000
    # Every stage's time, launches and algorithmic bandwidth, from the one
    # profiled step that chose the dominant kernel.
    out["stages"] = {k: {"ms": s["ms"], "launches": s["launches"],
                         "GBps": (s["bytes"] / (s["ms"] / 1000) / 1e9) if s["ms"] > 0 else None}
                     for k, s in stages.items() if s["launches"]}

    if args.compare_per_tree and args.workload == "c4":
        f = items[0][1]
        trees = []
        for b in range(f.B):
            v0, v1 = int(f.voff[b]), int(f.voff[b + 1])
            e0, e1 = v0 - b, v1 - b - 1
            u, v, w = calls[0][2][e0:e1], calls[0][3][e0:e1], calls[0][4][e0:e1]
            trees.append((v1 - v0, u, v, w, torch.empty(max(e1 - e0, 0), dtype=torch.int32, device=dev),
                          torch.empty(v1 - v0, dtype=torch.int32, device=dev)))

        def per_tree():
            for t in trees:
                st = pd.dendrogram_into(*t)
                if st != pd.OK:
                    raise RuntimeError(pd.status_string(st))
        per_tree()
        torch.cuda.synchronize()
        a = time.perf_counter()
        per_tree()
        torch.cuda.synchronize()
        per_s = time.perf_counter() - a
        out["per_tree_calls"] = {"seconds": per_s, "edges_per_s": total_edges / per_s,
                                 "batched_speedup": per_s / (ms_per_step / 1000.0), "calls": len(trees)}

    if any(kind == "flat" for kind, _ in items):
        out["metric"] = "MST edges/sec -> dendrogram + HDBSCAN* flat clusters"
        out["config"]["min_cluster_size"] = FLAT_MCS
        out["config"]["clusters"] = flat_k[-1] if flat_k else None
        if not args.no_cpu_baseline:
            flat_baseline(out)
        print(json.dumps(out), flush=True)
        return
    if not args.no_extras and args.workload == "c3":
        out["c4_batched"] = side_batched(dev)
        out["c5_serving_short"] = side_serving(dev)
        out["size_sweep"] = size_sweep(dev, items[0][1])
    if not args.no_cpu_baseline:
        oracle_baseline(out, items, args.workload)
    print(json.dumps(out), flush=True)


def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the share of the host given to one GPU)."""
    try:
        t = len(os.sched_getaffinity(0))
    except AttributeError:
        t = os.cpu_count() or 1
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return min(t, omp) if omp > 0 else t


def oracle_baseline(out, items, workload):
    """The CPU oracle on the step's own inputs, on this host: its (w, id)
    comparison sort on every host thread and on one, each timed apart from
    the sequential union-find sweep (the shape of the paper's multithreaded
    union-find comparison: a parallel sort, then a sequential sweep)."""
    import numpy as np
    import oracle
    threads = host_threads()
    total_edges = sum(obj.m if kind == "tree" else obj.m_total for kind, obj in items)
    runs = {}
    results = []
    for T in (threads, 1):
        log(f"timing the CPU oracle on the same inputs, {T} thread(s) ...")
        sort_s = sweep_s = 0.0
        t1 = time.perf_counter()
        res = []
        for kind, obj in items:
            if kind == "tree":
                ep, vp, a, b = oracle.dendrogram_timed(obj.n, obj.u, obj.v, obj.w, threads=T)
                sort_s += a
                sweep_s += b
                res.append((ep, vp))
            else:
                for bb in range(obj.B):
                    v0, v1 = int(obj.voff[bb]), int(obj.voff[bb + 1])
                    e0, e1 = v0 - bb, v1 - bb - 1
                    ep, vp, a, b = oracle.dendrogram_timed(v1 - v0, obj.u[e0:e1], obj.v[e0:e1], obj.w[e0:e1],
                                                           threads=T)
                    sort_s += a
                    sweep_s += b
                res.append(None)
        wall = time.perf_counter() - t1
        runs[T] = {"value": total_edges / wall, "seconds": wall, "sort_s": sort_s, "sweep_s": sweep_s}
        if T == 1:
            results = res
    # Imbalance (the paper's Table 2): dendrogram height over log2 n, from
    # the oracle's output (single trees).
    imb = []
    for (kind, obj), r in zip(items, results):
        if kind == "tree" and r is not None:
            h = oracle.dendrogram_height(r[0], r[1])
            imb.append({"n": obj.n, "height": h, "imb": h / math.log2(obj.n)})
    if imb:
        out["config"]["imbalance"] = imb
    # The multithreaded CPU form of the same method (single trees only),
    # checked against the oracle's output on the same inputs.
    if all(kind == "tree" for kind, _ in items):
        from paper_2401_06089_amd import cpu as pcpu
        t2 = time.perf_counter()
        mt = [pcpu.dendrogram(obj.n, obj.u, obj.v, obj.w, threads=threads) for _, obj in items]
        mt_s = time.perf_counter() - t2
        ok = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(mt, results))
        out["cpu_pandora_mt"] = {"value": total_edges / mt_s, "unit": "edges/s", "threads": threads,
                                 "seconds": mt_s, "matches_oracle": ok,
                                 "speedup_vs_oracle": runs[threads]["seconds"] / mt_s}
    par, one = runs[threads], runs[1]
    out["cpu_baseline"] = {
        "value": par["value"], "unit": "edges/s", "cores": threads, "kind": "oracle",
        "sample": f"one full step of {workload} ({total_edges} edges): comparison merge sort of (w, id) on "
                  f"{threads} host threads, then the sequential union-find sweep",
        "seconds": par["seconds"], "sort_s": par["sort_s"], "sweep_s": par["sweep_s"],
        "single_thread": {"value": one["value"], "seconds": one["seconds"], "sort_s": one["sort_s"],
                          "sweep_s": one["sweep_s"]},
        "host_cpu": cpu_model(), "host_threads_available": os.cpu_count(),
        "gpu_speedup_vs_oracle": out["value"] / par["value"],
    }


def side_batched(dev, reps=5):
    """The 4,096-tree forest (about 5e7 edges) in one batched call, against
    the same trees built one call per tree on the same stream."""
    import torch
    import gen
    import paper_2401_06089_amd as pd
    f = gen.c4_batched(0)
    u = torch.from_numpy(f.u).to(dev)
    v = torch.from_numpy(f.v).to(dev)
    w = torch.from_numpy(f.w).to(dev)
    pd.dendrogram_batched(f.voff, u, v, w)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = time.perf_counter()
        pd.dendrogram_batched(f.voff, u, v, w)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    batched = statistics.median(ts)
    trees = []
    for b in range(f.B):
        v0, v1 = int(f.voff[b]), int(f.voff[b + 1])
        e0, e1 = v0 - b, v1 - b - 1
        trees.append((v1 - v0, u[e0:e1], v[e0:e1], w[e0:e1],
                      torch.empty(max(e1 - e0, 0), dtype=torch.int32, device=dev),
                      torch.empty(v1 - v0, dtype=torch.int32, device=dev)))

    def per_tree():
        for t in trees:
            st = pd.dendrogram_into(*t)
            if st != pd.OK:
                raise RuntimeError(pd.status_string(st))
    per_tree()
    torch.cuda.synchronize()
    a = time.perf_counter()
    per_tree()
    torch.cuda.synchronize()
    per_s = time.perf_counter() - a
    del trees, u, v, w
    torch.cuda.empty_cache()
    return {"workload": "c4", "description": WORKLOADS["c4"], "trees": f.B, "edges": int(f.m_total),
            "batched_ms": 1000 * batched, "batched_edges_per_s": f.m_total / batched,
            "per_tree_calls_ms": 1000 * per_s, "per_tree_edges_per_s": f.m_total / per_s,
            "batched_speedup": per_s / batched, "reps": reps}


SWEEP_SIZES = (1_000, 10_000, 100_000, 1_000_000, 10_000_000, 50_000_000)


def size_sweep(dev, c3_tree=None, reps=5):
    """Problem-size sweep on the two single-tree shapes (random recursive tree
    with uniform weights; the preferential-attachment tree with lognormal
    weights and bridges): the GPU path (median of `reps` calls, each with the
    autotuned settings for its size) against the multithreaded CPU form of
    the same method on every host thread (one call), both on the same inputs.
    Shows where the GPU saturates and where it overtakes the CPU."""
    import numpy as np
    import torch
    import gen
    import paper_2401_06089_amd as pd
    from paper_2401_06089_amd import cpu as pcpu
    threads = host_threads()
    rows = []
    for shape in ("rrt", "pa"):
        for n in SWEEP_SIZES:
            if shape == "pa" and n == 50_000_000 and c3_tree is not None:
                t = c3_tree
            elif shape == "pa":
                t = gen.c3_pref_attach(0, n=n)
            else:
                t = gen.rrt(n, 0)
            u = torch.from_numpy(t.u).to(dev)
            v = torch.from_numpy(t.v).to(dev)
            w = torch.from_numpy(t.w).to(dev)
            ep = torch.empty(t.m, dtype=torch.int32, device=dev)
            vp = torch.empty(t.n, dtype=torch.int32, device=dev)
            for _ in range(2):
                st = pd.dendrogram_into(t.n, u, v, w, ep, vp)
                if st != pd.OK:
                    raise RuntimeError(pd.status_string(st))
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                a = time.perf_counter()
                pd.dendrogram_into(t.n, u, v, w, ep, vp)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - a)
            gpu_s = statistics.median(ts)
            a = time.perf_counter()
            cep, cvp = pcpu.dendrogram(t.n, t.u, t.v, t.w, threads=threads)
            cpu_s = time.perf_counter() - a
            same = bool(np.array_equal(cep, ep.cpu().numpy()) and np.array_equal(cvp, vp.cpu().numpy()))
            rows.append({"shape": shape, "n": t.n, "gpu_ms": 1000 * gpu_s, "gpu_edges_per_s": t.m / gpu_s,
                         "cpu_mt_ms": 1000 * cpu_s, "cpu_mt_edges_per_s": t.m / cpu_s,
                         "gpu_over_cpu_mt": cpu_s / gpu_s, "same_result": same})
            del u, v, w, ep, vp
    torch.cuda.empty_cache()
    return {"cpu_threads": threads, "host_cpu": cpu_model(), "rows": rows}


def side_serving(dev):
    """A short open-loop serving run (the c5 mix at 2,000 requests/s) from a
    smaller device pool."""
    ns = argparse.Namespace(rate=2000.0, duration=15.0, discard=3.0, pool=96, streams=2, budget_gb=200.0,
                            max_batch_edges=8_000_000, policy="small_first")
    r = run_serving(ns, dev, emit=False)
    return {"workload": "c5", "duration_s": ns.duration, "discarded_s": ns.discard, "pool_trees": ns.pool,
            "rate_per_s": ns.rate, "edges_per_s": r["value"], "latency_ms": r["latency_ms"],
            "requests": r["requests"]}


def uniform_points(n, dim, seed):
    import numpy as np
    import gen
    return gen.uniform_f64(n * dim, seed, 21).reshape(n, dim).astype(np.float32)


def run_points(args, dev):
    """HDBSCAN* on a point cloud: MST, dendrogram and flat clusters per step."""
    import numpy as np
    import torch

    import paper_2401_06089_amd as pd

    npts = args.points
    pts = torch.from_numpy(uniform_points(npts, HDB_DIM, 0)).to(dev)
    torch.cuda.synchronize()
    ks = []

    def step():
        lab, st = pd.hdbscan(pts, HDB_MIN_PTS, FLAT_MCS)
        ks.append(st.numel())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pd.profile_enable(pd.PROFILE_ALL)
    step()
    torch.cuda.synchronize()
    stages = pd.profile_read()
    pd.profile_enable(0)
    lat = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps
    search = stages["emst_search"]
    achieved = search["bytes"] / (search["ms"] / 1000.0) / 1e12 if search["ms"] > 0 else 0.0
    out = {
        "metric": "HDBSCAN* points/sec (mutual-reachability MST + dendrogram + flat clusters)",
        "value": npts * args.steps / elapsed,
        "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "hdb3d", "description": WORKLOADS["hdb3d"], "points": npts, "dim": HDB_DIM,
                   "min_pts": HDB_MIN_PTS, "min_cluster_size": FLAT_MCS, "clusters": ks[-1] if ks else None,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": 1000 * statistics.median(lat), "p99": 1000 * float(np.percentile(lat, 99)),
                       "per": "step"},
        "roofline": {"bound": "alu", "kernel": "emst_search", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": None, "ops": "fp64 operations of the point pairs the searches examine (3 per coordinate + 2), counted on the device in the profiled step",
                     "launches": search["launches"]},
        "stages": {k: {"ms": v["ms"], "launches": v["launches"]} for k, v in stages.items() if v["launches"]},
    }
    if not args.no_cpu_baseline:
        from oracle.emst import emst as oracle_emst
        from oracle.flat_clusters import flat_clusters as oracle_flat
        sample = uniform_points(4000, HDB_DIM, 0)
        log("timing the CPU oracle on a 4,000-point sample ...")
        t1 = time.perf_counter()
        u, v, _, w32, _ = oracle_emst(sample, HDB_MIN_PTS)
        oracle_flat(len(sample), u, v, w32, FLAT_MCS)
        cpu_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": len(sample) / cpu_s, "unit": "points/s", "cores": 1, "kind": "oracle",
                               "sample": "4,000 points of the same generator (the oracle is O(n^2), so its rate "
                                         "falls with n)",
                               "seconds": cpu_s, "host_cpu": cpu_model(), "host_threads_available": os.cpu_count()}
    print(json.dumps(out), flush=True)


def flat_baseline(out):
    """The oracle (dendrogram, then flat clusters) on a bounded sample: the
    same generator at 2,000,000 vertices."""
    import gen
    from oracle.flat_clusters import flat_clusters as oracle_flat
    sample = gen.c3_pref_attach(0, n=2_000_000)
    log("timing the CPU oracle on a 2,000,000-vertex sample ...")
    t1 = time.perf_counter()
    lab, st = oracle_flat(sample.n, sample.u, sample.v, sample.w, FLAT_MCS)
    cpu_s = time.perf_counter() - t1
    out["cpu_baseline"] = {"value": (sample.n - 1) / cpu_s, "unit": "edges/s", "cores": 1, "kind": "oracle",
                           "sample": "preferential-attachment tree of 2,000,000 vertices from the same "
                                     "generator (seed 0): oracle dendrogram (C) + flat clusters (Python)",
                           "seconds": cpu_s, "clusters": int(st.size), "host_cpu": cpu_model(),
                           "host_threads_available": os.cpu_count()}


def run_serving(args, dev, emit=True):
    """Open-loop serving run: Poisson arrivals, continuous batching, p50/p99 latency."""
    import numpy as np
    import torch

    import gen
    from paper_2401_06089_amd.serve import DendrogramServer, Request, latency_stats

    rng_sizes = gen.uniform_f64(args.pool, 0, stream=11)
    sizes = np.floor(np.exp(np.log(1e3) + rng_sizes * (np.log(1e7) - np.log(1e3)))).astype(np.int64)
    t0 = time.time()
    pool = []
    for i, n in enumerate(sizes):
        t = gen.rrt(int(n), gen.hash2(5, i), weights="lognormal")
        pool.append((t.n, torch.from_numpy(t.u).to(dev), torch.from_numpy(t.v).to(dev),
                     torch.from_numpy(t.w).to(dev)))
        if i % 64 == 63:
            log(f"pool: {i + 1}/{len(sizes)} trees")
    torch.cuda.synchronize()
    log(f"pool of {len(pool)} trees ({int(sizes.sum() - len(sizes))} edges) in {time.time() - t0:.1f}s")

    n_req = int(args.rate * args.duration * 1.2) + 16
    gaps = -np.log(1.0 - gen.uniform_f64(n_req, 0, stream=12)) / args.rate
    offsets = np.cumsum(gaps)
    offsets = offsets[offsets < args.duration]
    picks = (gen.uniform_f64(len(offsets), 0, stream=13) * len(pool)).astype(np.int64)

    srv = DendrogramServer(int(args.budget_gb * 1e9), streams=args.streams,
                           max_batch_edges=args.max_batch_edges, policy=args.policy)
    # warm the library and every stream's scratch once before the clock starts
    warm = [Request(-1 - k, *pool[int(np.argmax(sizes))], arrival=time.perf_counter())
            for k in range(args.streams)]
    for r in warm:
        srv.submit(r)
    for r in warm:
        r.future.result()
    with srv.cv:
        srv.done.clear()
        srv.batches = 0

    # The client consumes each result as it completes (here: checks it and
    # drops it), so device memory holds only what is in flight.
    done_cv = threading.Condition()
    done = {"n": 0, "failed": []}

    def consumed(r):
        def cb(f):
            exc = f.exception()
            r.future = None
            with done_cv:
                if exc is not None:
                    done["failed"].append((r.rid, repr(exc)))
                done["n"] += 1
                done_cv.notify_all()
        return cb

    # Python's cyclic garbage collector is paused for the timed window: its
    # full collections walk every live request record the client keeps for
    # the statistics (10^5 of them) and stall every thread, the server's
    # workers included, for tens of milliseconds.  Reference counting still
    # frees every result as soon as the client drops it.
    gc_was_enabled = gc.isenabled()
    gc.disable()
    start = time.perf_counter()
    reqs = []
    for i, off in enumerate(offsets):
        now = time.perf_counter()
        due = start + off
        if due > now:
            time.sleep(due - now)
        n, u, v, w = pool[int(picks[i])]
        r = Request(i, n, u, v, w, arrival=due)
        reqs.append(r)
        fut = srv.submit(r)
        fut.add_done_callback(consumed(r))
    with done_cv:
        while done["n"] < len(reqs):
            done_cv.wait(timeout=1.0)
    end = time.perf_counter()
    if gc_was_enabled:
        gc.enable()
    if done["failed"]:
        raise RuntimeError(f"{len(done['failed'])} requests failed, first: {done['failed'][0]}")
    srv.close()
    kept = [r for r in reqs if r.arrival - start >= args.discard]
    span = max(r.finished for r in kept) - min(r.arrival for r in kept) if kept else 1.0
    edges = sum(r.n - 1 for r in kept)
    stats = latency_stats(reqs, args.discard, start)
    out = {
        "metric": "MST edges/sec -> dendrogram (serving)",
        "value": edges / span,
        "unit": "edges/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "c5", "description": WORKLOADS["c5"], "rate_per_s": args.rate,
                   "duration_s": args.duration, "discarded_s": args.discard, "pool_trees": len(pool),
                   "streams": args.streams, "budget_bytes": srv.budget,
                   "max_batch_edges": args.max_batch_edges, "policy": args.policy},
        "latency_ms": {"p50": stats.get("p50_ms"), "p99": stats.get("p99_ms"),
                       "mean": stats.get("mean_ms"), "max": stats.get("max_ms"), "per": "request"},
        "requests": {"submitted": len(reqs), "measured": stats.get("count"),
                     "offered_edges_per_s": float(sum(pool[int(p)][0] - 1 for p in picks) / args.duration),
                     "batches": srv.batches, "requests_per_batch": len(reqs) / max(srv.batches, 1),
                     "max_concurrent_batches": srv.max_concurrent,
                     "reserved_bytes": srv.reserved, "peak_admitted_bytes": srv.peak_in_use,
                     "wall_s": end - start},
    }
    del pool
    torch.cuda.empty_cache()
    if emit:
        print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
