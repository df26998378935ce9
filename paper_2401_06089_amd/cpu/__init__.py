"""Multithreaded CPU form of the dendrogram path (OpenMP), beside the GPU
library: the same method on host arrays, for hosts without a GPU and for
comparing the two.  The GPU binding never calls it.

    from paper_2401_06089_amd import cpu
    ep, vp = cpu.dendrogram(n, u, v, w, threads=16)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpandora_cpu.so")
_lib = None


def build() -> str:
    src = os.path.join(_HERE, "pandora_cpu.cpp")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fvisibility=hidden",
                           "-Wall", "-o", tmp, src])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2401_06089_amd.cpu.build()")
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        lib.pandora_cpu_dendrogram.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_int]
        lib.pandora_cpu_dendrogram.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def dendrogram_status(n: int, u, v, w, threads: int = 0):
    """(status, edge_parent, vertex_parent); status codes as the GPU library's."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    ep = np.empty(max(n - 1, 0), np.int32)
    vp = np.empty(max(n, 0), np.int32)
    st = _load().pandora_cpu_dendrogram(int(n), _p(u), _p(v), _p(w), _p(ep), _p(vp), int(threads))
    return st, ep, vp


def dendrogram(n: int, u, v, w, threads: int = 0):
    st, ep, vp = dendrogram_status(n, u, v, w, threads)
    if st != 0:
        raise RuntimeError(f"pandora cpu status {st}")
    return ep, vp
