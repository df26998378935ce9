"""Continuous-batching request server for dendrogram builds on one GPU.

Requests (one tree each, device-resident u, v, w) wait in a queue.  Each of S
slots owns a worker thread, a HIP stream, a caller-owned library workspace and
an input arena, allocated once and sized for the largest batch; the byte
budget covers those reservations plus the outputs of every admitted request,
so it bounds the device memory the server uses.

A free slot takes the waiting requests that fit (budget, edge cap, tree cap;
in arrival order, or smallest first behind the oldest), copies their inputs
into its arena (one copy kernel per array; a lone request is read in place)
and builds all their dendrograms with one batched call on its stream.
Requests that arrive while the slots are busy wait and are admitted together
as slots free up, so batches grow with the load, and batches on different
slots overlap on the device.  The batched call picks its level loop by size
(exact grids with a small read-back per level for large batches, the
host-free loop below the tuned threshold), which measured faster here than
the stream-ordered call for every batch: the host-free loop has to size
every grid by the level bounds.  A forest call gives every tree exactly the
result it gets alone, so a request's answer does not depend on what it was
batched with.  If a batch reports an input error, its requests are rebuilt
one by one so that the error reaches only the request that caused it.
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

from . import PandoraError, dendrogram, dendrogram_batched, set_workspace, workspace_bytes


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
    stream: Optional[torch.cuda.Stream] = None  # the submitting stream (receives the outputs)
    future: Future = field(default_factory=Future)
    admitted: float = 0.0
    started: float = 0.0
    finished: float = 0.0


def request_footprint(n: int) -> int:
    """Device bytes one admitted request holds until its client drops the
    result: its outputs (edge_parent and vertex_parent).  Scratch and input
    arenas belong to the slots and are reserved once."""
    return 4 * (n - 1) + 4 * n


def slot_bytes(max_edges: int, max_trees: int) -> int:
    """Bytes one slot reserves: the library workspace for any batch of at most
    max_edges edges over max_trees trees, plus the u, v, w input arena."""
    return workspace_bytes(max_edges + max_trees, max_trees) + 12 * max_edges


@dataclass
class _Slot:
    stream: torch.cuda.Stream
    workspace: torch.Tensor
    u: torch.Tensor
    v: torch.Tensor
    w: torch.Tensor
    busy: bool = False


class DendrogramServer:
    def __init__(self, budget_bytes: int, streams: int = 2, max_batch_edges: int = 8 << 20,
                 device: int = 0, policy: str = "small_first", max_batch_trees: int = 4096,
                 max_tree_vertices: int = 1 << 24):
        if policy not in ("fifo", "small_first"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy = policy
        self.budget = int(budget_bytes)
        self.max_batch_edges = int(max_batch_edges)
        self.max_batch_trees = int(max_batch_trees)
        # a lone request may exceed the batch edge cap, up to the largest tree
        # the slots are sized for
        self.max_tree_vertices = int(max_tree_vertices)
        self.slot_edges = max(self.max_batch_edges, self.max_tree_vertices - 1)
        self.device = torch.device("cuda", device)
        self.pending: collections.deque[Request] = collections.deque()
        self.cv = threading.Condition()
        self.in_use = 0
        self.peak_in_use = 0
        self.closed = False
        self.done: List[Request] = []
        self.batches = 0
        self.max_concurrent = 0
        self._running = 0
        self.slots: List[_Slot] = []
        per_slot = slot_bytes(self.slot_edges, self.max_batch_trees) if streams > 0 else 0
        self.reserved = per_slot * streams
        if self.reserved > self.budget:
            raise ValueError(f"{streams} slots need {self.reserved} bytes, budget is {self.budget}")
        for _ in range(streams):
            with torch.cuda.device(self.device):
                st = torch.cuda.Stream(device=self.device)
                ws = torch.empty(per_slot - 12 * self.slot_edges, dtype=torch.uint8, device=self.device)
                set_workspace(ws, stream=st)
                self.slots.append(_Slot(st, ws,
                                        torch.empty(self.slot_edges, dtype=torch.int32, device=self.device),
                                        torch.empty(self.slot_edges, dtype=torch.int32, device=self.device),
                                        torch.empty(self.slot_edges, dtype=torch.float32, device=self.device)))
        self.threads = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in self.slots]
        for t in self.threads:
            t.start()

    # ---- client side ------------------------------------------------------------
    def submit(self, req: Request) -> Future:
        """Queue one tree.  Its tensors may still be being written by work on the
        submitting thread's current stream: the slot's stream waits for that
        work before reading them, and the outputs are tied to that stream."""
        req.footprint = request_footprint(req.n)
        if isinstance(req.w, torch.Tensor) and req.w.is_cuda:
            req.stream = torch.cuda.current_stream(self.device)
            req.ready = torch.cuda.Event()
            req.ready.record(req.stream)
        with self.cv:
            if self.closed:
                req.future.set_exception(RuntimeError("the server is closed"))
                return req.future
            if req.footprint + self.reserved > self.budget:
                req.future.set_exception(MemoryError(
                    f"request {req.rid} needs {req.footprint} bytes beyond the {self.reserved} reserved, "
                    f"budget is {self.budget}"))
                return req.future
            if req.n > self.max_tree_vertices:
                req.future.set_exception(MemoryError(
                    f"request {req.rid} has {req.n} vertices, the slots hold trees of at most "
                    f"{self.max_tree_vertices}"))
                return req.future
            self.pending.append(req)
            self.cv.notify_all()
        return req.future

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        for s in self.slots:
            set_workspace(None, stream=s.stream)

    # ---- batching policy ------------------------------------------------------------
    def _take_batch(self) -> Optional[List[Request]]:
        """Under the lock: admit waiting requests while they fit the byte budget,
        the batch edge cap and the tree cap.  "fifo" takes them in arrival
        order and stops at the first that does not fit; "small_first" takes
        the smallest waiting requests first (the oldest request always heads
        the batch, so none waits behind an endless stream of smaller ones)."""
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
            if batch and (edges + (r.n - 1) > self.max_batch_edges or len(batch) >= self.max_batch_trees):
                if self.policy == "fifo":
                    break
                continue
            if self.reserved + self.in_use + r.footprint > self.budget:
                break
            self.in_use += r.footprint
            self.peak_in_use = max(self.peak_in_use, self.reserved + self.in_use)
            r.admitted = time.perf_counter()
            batch.append(r)
            taken.append(i)
            edges += r.n - 1
        if taken:
            keep = set(taken)
            self.pending = collections.deque(r for i, r in enumerate(self.pending) if i not in keep)
        return batch or None

    # ---- slot workers ------------------------------------------------------------------
    def _worker(self, slot: _Slot):
        torch.cuda.set_device(self.device)
        while True:
            with self.cv:
                while True:
                    batch = self._take_batch()
                    if batch is not None or (self.closed and not self.pending):
                        break
                    self.cv.wait(timeout=0.05)
                if batch is None:
                    return
                slot.busy = True
                self._running += 1
                self.max_concurrent = max(self.max_concurrent, self._running)
            try:
                self._run_batch(slot, batch)
            except Exception as e:   # surface the failure on every request of the batch
                for r in batch:
                    if not r.future.done():
                        r.future.set_exception(e)
            finally:
                with self.cv:
                    slot.busy = False
                    self._running -= 1
                    self.batches += 1
                    for r in batch:
                        self.in_use -= r.footprint
                    self.done.extend(batch)
                    self.cv.notify_all()

    def _run_batch(self, slot: _Slot, batch: List[Request]):
        start = time.perf_counter()
        sizes = np.array([r.n for r in batch], dtype=np.int64)
        voff = np.zeros(len(batch) + 1, dtype=np.int64)
        np.cumsum(sizes, out=voff[1:])
        E = int(voff[-1]) - len(batch)
        with torch.cuda.stream(slot.stream):
            for r in batch:
                if r.ready is not None:
                    slot.stream.wait_event(r.ready)
            if len(batch) == 1:
                u, v, w = batch[0].u, batch[0].v, batch[0].w
            else:
                u, v, w = slot.u[:E], slot.v[:E], slot.w[:E]
                torch.cat([r.u for r in batch], out=u)
                torch.cat([r.v for r in batch], out=v)
                torch.cat([r.w for r in batch], out=w)
            try:
                ep, vp = dendrogram_batched(voff, u, v, w, stream=slot.stream)
                results = [(ep[int(voff[b]) - b:int(voff[b + 1]) - b - 1], vp[int(voff[b]):int(voff[b + 1])])
                           for b in range(len(batch))]
            except PandoraError:
                # an input error somewhere in the batch: rebuild each tree alone
                results = []
                for r in batch:
                    try:
                        results.append(dendrogram(r.u, r.v, r.w, n=r.n, stream=slot.stream))
                    except PandoraError as e:
                        results.append(e)
        finished = time.perf_counter()
        for r, res in zip(batch, results):
            r.started = start
            r.finished = finished
            if isinstance(res, Exception):
                r.future.set_exception(res)
                continue
            if r.stream is not None:   # the client's stream may still use them when it drops them
                for t in res:
                    t.record_stream(r.stream)
            r.future.set_result(res)


def latency_stats(reqs: List[Request], warmup_s: float, t0: float) -> dict:
    lat = np.array([r.finished - r.arrival for r in reqs if r.arrival - t0 >= warmup_s])
    if lat.size == 0:
        return {"count": 0}
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
