"""Continuous-batching request server for dendrogram builds on one GPU.

Requests (one tree each, device-resident u, v, w) are admitted by their HBM
footprint against a byte budget: the library's scratch bytes for the tree
(``pandora_workspace_bytes``) plus its inputs and outputs.  Each of S worker
threads owns a HIP stream.  When a worker is free it takes every admitted
request that is waiting (up to an edge cap), concatenates them into one
forest on its stream, builds all their dendrograms with one batched call,
hands each request its slice of the outputs, and releases the bytes.
Requests that arrive while other batches run are admitted as bytes free up,
and batches on different streams overlap on the device.  A forest call gives
every tree exactly the result it gets alone, so a request's answer does not
depend on what it was batched with.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import dendrogram_batched, workspace_bytes


@dataclass
class Request:
    rid: int
    n: int
    u: torch.Tensor
    v: torch.Tensor
    w: torch.Tensor
    arrival: float                     # scheduled arrival (perf_counter seconds)
    footprint: int = 0
    ready: Optional[torch.cuda.Event] = None   # inputs written (recorded at submit)
    future: Future = field(default_factory=Future)
    admitted: float = 0.0
    started: float = 0.0
    finished: float = 0.0


def request_footprint(n: int) -> int:
    """HBM bytes one tree occupies while it is built: scratch + inputs + outputs."""
    io = 12 * (n - 1) + 4 * (n - 1) + 4 * n
    return workspace_bytes(n, 1) + io


class DendrogramServer:
    def __init__(self, budget_bytes: int, streams: int = 4, max_batch_edges: int = 64 << 20,
                 device: int = 0, policy: str = "fifo"):
        if policy not in ("fifo", "small_first"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy = policy
        self.peak_in_use = 0
        self.budget = int(budget_bytes)
        self.max_batch_edges = int(max_batch_edges)
        self.device = torch.device("cuda", device)
        self.pending: collections.deque[Request] = collections.deque()
        self.cv = threading.Condition()
        self.in_use = 0
        self.closed = False
        self.done: List[Request] = []
        self.batches = 0
        self.max_concurrent = 0
        self._running = 0
        self.workers = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                        for i in range(streams)]
        for t in self.workers:
            t.start()

    # ---- client side ------------------------------------------------------------
    def submit(self, req: Request) -> Future:
        """Queue one tree.  Its tensors may still be being written by work on the
        submitting thread's current stream: the worker's stream waits for that
        work before reading them."""
        req.footprint = request_footprint(req.n)
        if isinstance(req.w, torch.Tensor) and req.w.is_cuda:
            req.ready = torch.cuda.Event()
            req.ready.record(torch.cuda.current_stream(self.device))
        with self.cv:
            if self.closed:
                req.future.set_exception(RuntimeError("the server is closed"))
                return req.future
            if req.footprint > self.budget:
                req.future.set_exception(MemoryError(
                    f"request {req.rid} needs {req.footprint} bytes, budget is {self.budget}"))
                return req.future
            self.pending.append(req)
            self.cv.notify_all()
        return req.future

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self.workers:
            t.join()

    # ---- workers -----------------------------------------------------------------
    def _take_batch(self) -> Optional[List[Request]]:
        """Under the lock: admit waiting requests while they fit the byte budget
        and the batch edge cap.  "fifo" takes them in arrival order and stops at
        the first that does not fit; "small_first" takes the smallest waiting
        requests first (the oldest request always heads the batch, so none
        waits behind an endless stream of smaller ones)."""
        if not self.pending:
            return None
        if self.policy == "fifo":
            order = list(range(len(self.pending)))
        else:
            rest = sorted(range(1, len(self.pending)), key=lambda i: self.pending[i].n)
            order = [0] + rest
        batch: List[Request] = []
        taken = []
        edges = 0
        for i in order:
            r = self.pending[i]
            if batch and edges + (r.n - 1) > self.max_batch_edges:
                if self.policy == "fifo":
                    break
                continue
            if self.in_use + r.footprint > self.budget:
                break
            self.in_use += r.footprint
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            r.admitted = time.perf_counter()
            batch.append(r)
            taken.append(i)
            edges += r.n - 1
        if taken:
            keep = set(taken)
            self.pending = collections.deque(r for i, r in enumerate(self.pending) if i not in keep)
        return batch or None

    def _worker(self, idx: int):
        torch.cuda.set_device(self.device)
        stream = torch.cuda.Stream(device=self.device)
        while True:
            with self.cv:
                batch = None
                while True:
                    batch = self._take_batch()
                    if batch is not None or (self.closed and not self.pending):
                        break
                    self.cv.wait(timeout=0.05)
                if batch is None:
                    return
                self._running += 1
                self.max_concurrent = max(self.max_concurrent, self._running)
            try:
                self._run_batch(batch, stream)
            except Exception as e:   # surface the failure on every request of the batch
                for r in batch:
                    if not r.future.done():
                        r.future.set_exception(e)
            finally:
                with self.cv:
                    self._running -= 1
                    self.batches += 1
                    for r in batch:
                        self.in_use -= r.footprint
                    self.cv.notify_all()

    def _run_batch(self, batch: List[Request], stream: torch.cuda.Stream):
        start = time.perf_counter()
        sizes = np.array([r.n for r in batch], dtype=np.int64)
        voff = np.zeros(len(batch) + 1, dtype=np.int64)
        np.cumsum(sizes, out=voff[1:])
        with torch.cuda.stream(stream):
            for r in batch:
                if r.ready is not None:
                    stream.wait_event(r.ready)
            if len(batch) == 1:
                u, v, w = batch[0].u, batch[0].v, batch[0].w
            else:
                u = torch.cat([r.u for r in batch])
                v = torch.cat([r.v for r in batch])
                w = torch.cat([r.w for r in batch])
            ep, vp = dendrogram_batched(voff, u, v, w, stream=stream)
        finished = time.perf_counter()
        for b, r in enumerate(batch):
            v0, v1 = int(voff[b]), int(voff[b + 1])
            r.started = start
            r.finished = finished
            r.future.set_result((ep[v0 - b:v1 - b - 1], vp[v0:v1]))
        with self.cv:
            self.done.extend(batch)


def latency_stats(reqs: List[Request], warmup_s: float, t0: float) -> dict:
    lat = np.array([r.finished - r.arrival for r in reqs if r.arrival - t0 >= warmup_s])
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
