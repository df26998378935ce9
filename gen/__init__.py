"""Seeded synthetic trees shared by the tests, the CPU oracle and the benchmark.

This module holds no dendrogram arithmetic: it draws tree shapes and edge
weights only (the C code in ``gen.c``, loaded with ctypes).  The paper's
datasets (Table 2) are not available; these synthetic shapes stand in for
them and span its range of dendrogram skew (its "Imb" column, 43 to 6e5):

* random recursive trees with fp32 uniform weights (mildly skewed),
* caterpillars whose spine weights rise along the path (heavily skewed),
* preferential-attachment trees with lognormal weights and 10x bridges
  (hub-dominated, like HDBSCAN* minimum spanning trees),
* adversarial closed forms: monotone path, star, constant weights,
  bit-reversal path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64


def build() -> str:
    """Compile gen.c into libgen.so next to it (plain gcc, no GPU)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gen_weights_uniform.argtypes = [_i64, _u64, _f32p]
    lib.gen_weights_lognormal.argtypes = [_i64, _u64, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_float, _f32p]
    lib.gen_rrt.argtypes = [_i64, _u64, _i32p, _i32p]
    lib.gen_pref_attach.argtypes = [_i64, _u64, _i32p, _i32p, _i32p]
    lib.gen_caterpillar.argtypes = [_i64, _i64, ctypes.c_double, _u64, _i32p, _i32p, _f32p]
    lib.gen_path.argtypes = [_i64, _i32p, _i32p]
    lib.gen_star.argtypes = [_i64, _i32p, _i32p]
    lib.gen_shuffle.argtypes = [_i64, _u64, _i32p, _i32p, _f32p, _i32p]
    lib.gen_uniform_f64.argtypes = [_i64, _u64, _u64, _f64p]
    lib.gen_normal_f64.argtypes = [_i64, _u64, _u64, _f64p]
    lib.gen_hash2.argtypes = [_u64, _u64]
    lib.gen_hash2.restype = _u64
    for f in ("gen_weights_uniform", "gen_weights_lognormal", "gen_rrt", "gen_pref_attach",
              "gen_caterpillar", "gen_path", "gen_star", "gen_shuffle", "gen_uniform_f64",
              "gen_normal_f64"):
        getattr(lib, f).restype = None
    _lib = lib
    return lib


class Tree:
    """n vertices, n-1 edges (u[i], v[i], w[i]); host numpy arrays."""

    __slots__ = ("n", "u", "v", "w", "name")

    def __init__(self, n, u, v, w, name=""):
        self.n = int(n)
        self.u = np.ascontiguousarray(u, dtype=np.int32)
        self.v = np.ascontiguousarray(v, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.float32)
        self.name = name

    @property
    def m(self) -> int:
        return self.n - 1


# ---- raw draws -------------------------------------------------------------

def uniform_f64(k: int, seed: int, stream: int = 4) -> np.ndarray:
    out = np.empty(k, np.float64)
    _load().gen_uniform_f64(k, seed, stream, out)
    return out


def normal_f64(k: int, seed: int, stream: int = 5) -> np.ndarray:
    out = np.empty(k, np.float64)
    _load().gen_normal_f64(k, seed, stream, out)
    return out


def hash2(a: int, b: int) -> int:
    return int(_load().gen_hash2(a, b))


# ---- weights ---------------------------------------------------------------

def weights_uniform(m: int, seed: int) -> np.ndarray:
    w = np.empty(max(m, 0), np.float32)
    if m > 0:
        _load().gen_weights_uniform(m, seed, w)
    return w


def weights_lognormal(m: int, seed: int, mu: float = 0.0, sigma: float = 1.5,
                      bridge_p: float = 0.0, bridge_mul: float = 10.0) -> np.ndarray:
    w = np.empty(max(m, 0), np.float32)
    if m > 0:
        _load().gen_weights_lognormal(m, seed, mu, sigma, bridge_p, bridge_mul, w)
    return w


# ---- shapes ----------------------------------------------------------------

def rrt(n: int, seed: int = 0, weights: str = "uniform") -> Tree:
    """Random recursive tree; fp32 uniform [0,1) (or lognormal(0,1.5)) weights."""
    m = n - 1
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    if m > 0:
        _load().gen_rrt(n, seed, u, v)
    w = weights_uniform(m, seed) if weights == "uniform" else weights_lognormal(m, seed)
    return Tree(n, u, v, w, f"rrt{n}")


def pref_attach(n: int, seed: int = 0, sigma: float = 1.5, bridge_p: float = 0.05,
                bridge_mul: float = 10.0) -> Tree:
    """Preferential attachment (p ~ deg+1), lognormal(0, sigma) fp32 weights,
    a fraction bridge_p of edges multiplied by bridge_mul."""
    m = n - 1
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    if m > 0:
        scratch = np.empty(2 * m, np.int32)
        _load().gen_pref_attach(n, seed, u, v, scratch)
        del scratch
    w = weights_lognormal(m, seed, 0.0, sigma, bridge_p, bridge_mul)
    return Tree(n, u, v, w, f"pa{n}")


def caterpillar(n: int, spine: int | None = None, noise: float = 1e-3, seed: int = 0) -> Tree:
    """Path of `spine` vertices (default 90% of n) plus leaves at random spine
    positions; weights rise along the spine with fp32 uniform noise."""
    if spine is None:
        spine = max(1, (9 * n) // 10)
    m = n - 1
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    w = np.empty(m, np.float32)
    if m > 0:
        _load().gen_caterpillar(n, spine, noise, seed, u, v, w)
    return Tree(n, u, v, w, f"caterpillar{n}")


def path(n: int, w: np.ndarray) -> Tree:
    m = n - 1
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    if m > 0:
        _load().gen_path(n, u, v)
    return Tree(n, u, v, w, f"path{n}")


def path_mono(n: int) -> Tree:
    """Path whose weights rise strictly along it: one chain of height n-1 and
    the deepest possible contraction pointers."""
    return path(n, np.arange(n - 1, dtype=np.float32))


def path_bitrev(levels: int) -> Tree:
    """Path of n = 2^levels vertices whose edge k = (k, k+1) has weight
    n - bitreverse(k+1): in every dyadic block the edge with the most trailing
    zeros is the heaviest, so the dendrogram is a perfect binary tree."""
    n = 1 << levels
    k = np.arange(1, n, dtype=np.int64)
    rev = np.zeros_like(k)
    for b in range(levels):
        rev |= ((k >> b) & 1) << (levels - 1 - b)
    return path(n, (n - rev).astype(np.float32))


def star(n: int, seed: int = 0) -> Tree:
    m = n - 1
    u = np.empty(m, np.int32)
    v = np.empty(m, np.int32)
    if m > 0:
        _load().gen_star(n, u, v)
    return Tree(n, u, v, weights_uniform(m, seed), f"star{n}")


def shuffled(t: Tree, seed: int) -> Tree:
    """Same tree with vertex labels permuted, edges reordered and each edge's
    orientation flipped at random."""
    u, v, w = t.u.copy(), t.v.copy(), t.w.copy()
    if t.m > 0:
        scratch = np.empty(t.n, np.int32)
        _load().gen_shuffle(t.n, seed, u, v, w, scratch)
    return Tree(t.n, u, v, w, t.name + "_shuf")


# ---- the measured workloads ------------------------------------------------

def c1_rrt(seed: int = 0) -> Tree:
    """Random recursive tree, n = 100,000, fp32 uniform weights."""
    return rrt(100_000, seed)


def c2a_rrt(seed: int = 0, n: int = 10_000_000) -> Tree:
    return rrt(n, seed)


def c2b_caterpillar(seed: int = 0, n: int = 10_000_000) -> Tree:
    """Caterpillar, 9,000,000-vertex spine plus 1,000,000 leaves (scaled with n)."""
    return caterpillar(n, (9 * n) // 10, 1e-3, seed)


def c3_pref_attach(seed: int = 0, n: int = 50_000_000) -> Tree:
    """HDBSCAN*-like tree: preferential attachment, lognormal(0, 1.5) weights,
    5% of edges x10 (bridges)."""
    return pref_attach(n, seed, 1.5, 0.05, 10.0)


class Forest:
    """B trees concatenated: tree b owns vertices [voff[b], voff[b+1]) and edges
    [voff[b]-b, voff[b+1]-b-1); u, v hold tree-local vertex ids."""

    __slots__ = ("voff", "u", "v", "w", "shapes")

    def __init__(self, voff, u, v, w, shapes=None):
        self.voff = np.ascontiguousarray(voff, dtype=np.int64)
        self.u = np.ascontiguousarray(u, dtype=np.int32)
        self.v = np.ascontiguousarray(v, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.float32)
        self.shapes = shapes

    @property
    def B(self) -> int:
        return len(self.voff) - 1

    @property
    def n_total(self) -> int:
        return int(self.voff[-1])

    @property
    def m_total(self) -> int:
        return self.n_total - self.B

    def tree(self, b: int) -> Tree:
        v0, v1 = int(self.voff[b]), int(self.voff[b + 1])
        e0, e1 = v0 - b, v1 - b - 1
        return Tree(v1 - v0, self.u[e0:e1], self.v[e0:e1], self.w[e0:e1], f"tree{b}")


def forest_from_trees(trees) -> Forest:
    sizes = np.array([t.n for t in trees], dtype=np.int64)
    voff = np.zeros(len(trees) + 1, np.int64)
    np.cumsum(sizes, out=voff[1:])
    cat = lambda xs, dt: (np.concatenate(xs) if len(xs) else np.empty(0, dt)).astype(dt)
    return Forest(voff, cat([t.u for t in trees], np.int32), cat([t.v for t in trees], np.int32),
                  cat([t.w for t in trees], np.float32), [t.name for t in trees])


def lognormal_sizes(B: int, seed: int, target_edges: int, sigma: float = 1.5,
                    lo: int = 100, hi: int = 1_000_000) -> np.ndarray:
    """B tree sizes clip(round(exp(mu + sigma z)), lo, hi) with mu set by
    bisection so that the edge total is as close as possible to target_edges."""
    z = normal_f64(B, seed, stream=6)

    def sizes(mu):
        return np.clip(np.rint(np.exp(mu + sigma * z)), lo, hi).astype(np.int64)

    a, b = 0.0, 20.0
    for _ in range(100):
        mid = 0.5 * (a + b)
        if int((sizes(mid) - 1).sum()) < target_edges:
            a = mid
        else:
            b = mid
    return sizes(b)


def c4_batched(seed: int = 0, B: int = 4096, target_edges: int = 50_000_000,
               hi: int = 1_000_000) -> Forest:
    """B trees with lognormal sizes in [100, hi], half random-recursive and half
    caterpillar (90% spine), fp32 uniform weights; ~target_edges edges total."""
    sz = lognormal_sizes(B, seed, target_edges, hi=hi)
    coin = uniform_f64(B, seed, stream=7)
    trees = []
    for b in range(B):
        s = hash2(seed, b)
        if coin[b] < 0.5:
            trees.append(rrt(int(sz[b]), s))
        else:
            trees.append(caterpillar(int(sz[b]), None, 1e-3, s))
    return forest_from_trees(trees)
