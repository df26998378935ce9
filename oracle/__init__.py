"""CPU oracle for the single-linkage dendrogram of a minimum spanning tree.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
loads it, and the two share no code.

``oracle.c`` is the bottom-up union-find construction (paper, Section
2.3.2): edges are visited in ascending (weight, id) order and each one
becomes the parent of the two clusters it merges.  ``checks.py`` holds the
independent checks that pin it (brute force, closed forms, invariants).
``flat_clusters.py`` takes HDBSCAN* flat clusters from that dendrogram
(pinned by ``tests/test_flat_oracle.py``), and ``emst.py`` builds the
mutual-reachability MST of a point cloud that HDBSCAN* starts from (pinned by
``tests/test_emst_oracle.py``).

Status codes: 0 ok, 1 invalid argument, 2 not a tree, 3 NaN weight,
6 vertex id out of range.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, INVALID_ARG, NOT_A_TREE, NAN_WEIGHT, BAD_VERTEX = 0, 1, 2, 3, 6

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile oracle.c into liboracle.so next to it (plain gcc)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-pthread", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_dendrogram.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_dendrogram.restype = ctypes.c_int
    lib.oracle_edge_order.argtypes = [ctypes.c_int64, _f32p, _i32p]
    lib.oracle_edge_order.restype = ctypes.c_int
    lib.oracle_dendrogram_batched.argtypes = [ctypes.c_int32, _i64p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_dendrogram_batched.restype = ctypes.c_int
    lib.oracle_dendrogram_mt.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.oracle_dendrogram_mt.restype = ctypes.c_int
    lib.oracle_edge_order_mt.argtypes = [ctypes.c_int64, _f32p, _i32p, ctypes.c_int]
    lib.oracle_edge_order_mt.restype = ctypes.c_int
    lib.oracle_dendrogram_height.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_dendrogram_height.restype = ctypes.c_int64
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def edge_order(w: np.ndarray, threads: int = 1) -> np.ndarray:
    """Edge ids sorted ascending by (w, id) (a merge sort on `threads` host threads)."""
    w = np.ascontiguousarray(w, dtype=np.float32)
    out = np.empty(len(w), np.int32)
    st = _load().oracle_edge_order_mt(len(w), w, out, int(threads))
    if st:
        raise OracleError(st)
    return out


def dendrogram_status(n, u, v, w):
    """(status, edge_parent, vertex_parent) for one tree."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    ep = np.empty(max(n - 1, 0), np.int32)
    vp = np.empty(max(n, 0), np.int32)
    st = _load().oracle_dendrogram(int(n), _ptr(u), _ptr(v), _ptr(w), _ptr(ep),
                                   vp.ctypes.data_as(ctypes.c_void_p) if vp.size else None)
    return st, ep, vp


def dendrogram(n, u, v, w):
    """(edge_parent, vertex_parent) of one tree; raises OracleError on bad input."""
    st, ep, vp = dendrogram_status(n, u, v, w)
    if st:
        raise OracleError(st)
    return ep, vp


def dendrogram_timed(n, u, v, w, threads: int = 1):
    """(edge_parent, vertex_parent, sort_seconds, sweep_seconds) of one tree:
    the (w, id) sort on `threads` host threads, then the sequential union-find
    sweep, each timed inside the C code."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    ep = np.empty(max(n - 1, 0), np.int32)
    vp = np.empty(max(n, 0), np.int32)
    ts, tw = ctypes.c_double(0.0), ctypes.c_double(0.0)
    st = _load().oracle_dendrogram_mt(int(n), _ptr(u), _ptr(v), _ptr(w), _ptr(ep),
                                      vp.ctypes.data_as(ctypes.c_void_p) if vp.size else None, int(threads),
                                      ctypes.byref(ts), ctypes.byref(tw))
    if st:
        raise OracleError(st)
    return ep, vp, ts.value, tw.value


def dendrogram_batched(voff, u, v, w):
    """Tree-local (edge_parent, vertex_parent) of a forest given by vertex offsets."""
    voff = np.ascontiguousarray(voff, dtype=np.int64)
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    B = len(voff) - 1
    N = int(voff[-1])
    ep = np.empty(max(N - B, 0), np.int32)
    vp = np.empty(N, np.int32)
    bad = ctypes.c_int32(-1)
    st = _load().oracle_dendrogram_batched(B, voff, _ptr(u), _ptr(v), _ptr(w), _ptr(ep),
                                           _ptr(vp), ctypes.byref(bad))
    if st:
        raise OracleError(st)
    return ep, vp


def dendrogram_height(edge_parent, vertex_parent) -> int:
    """Largest number of edge nodes from a vertex up to the root (the paper's
    imbalance is this over log2 n)."""
    ep = np.ascontiguousarray(edge_parent, dtype=np.int32)
    vp = np.ascontiguousarray(vertex_parent, dtype=np.int32)
    h = _load().oracle_dendrogram_height(len(vp), _ptr(ep), _ptr(vp))
    if h < 0:
        raise OracleError(1)
    return int(h)
