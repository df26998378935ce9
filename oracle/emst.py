"""CPU oracle for the mutual-reachability minimum spanning tree of a point
cloud (the input HDBSCAN* hands to the dendrogram).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
loads it, and the two share no code.

The paper's HDBSCAN* section builds this tree (with ArborX) before the
dendrogram; the definitions are HDBSCAN*'s (Campello et al. 2015):

* Points are fp32 coordinates, widened to fp64.  The squared distance of
  points i and j is the sum over coordinates k = 0, 1, ... (in that order)
  of (x_ik - x_jk)^2, each subtraction, square and addition rounded to fp64
  on its own (no fused multiply-add).
* Core distance (squared) of i for min_pts: its (min_pts - 1)-th smallest
  squared distance to another point (0 for min_pts = 1), i.e. counting the
  point itself among its min_pts nearest, as HDBSCAN* does.
* Mutual reachability (squared): max(core2(i), core2(j), d2(i, j)).
* Edges are totally ordered by (mutual reachability squared, min(i, j),
  max(i, j)); the minimum spanning tree under that order is unique.  Its
  edges come out in that order, with fp64 weight sqrt(mrd2) (correctly
  rounded) and its fp32 rounding for the dendrogram.

Prim's algorithm on the complete graph (O(n^2) memory-free sweeps) builds it.
"""
from __future__ import annotations

import numpy as np


def squared_distances_to(x: np.ndarray, i: int) -> np.ndarray:
    """d2(i, j) for every j, coordinates summed in order, no fused operations."""
    acc = np.zeros(x.shape[0], np.float64)
    for k in range(x.shape[1]):
        t = x[:, k] - x[i, k]
        acc = acc + t * t
    return acc


def core_distances2(points, min_pts: int) -> np.ndarray:
    x = np.asarray(points, np.float32).astype(np.float64)
    n = x.shape[0]
    if min_pts < 1 or n < min_pts:
        raise ValueError("need 1 <= min_pts <= n")
    core2 = np.zeros(n, np.float64)
    if min_pts == 1:
        return core2
    for i in range(n):
        d2 = squared_distances_to(x, i)
        d2[i] = np.inf
        core2[i] = np.partition(d2, min_pts - 2)[min_pts - 2]
    return core2


def emst(points, min_pts: int):
    """(u int32, v int32, w64 float64, w32 float32, mrd2 float64) of the n-1
    tree edges in ascending (mrd2, u, v) order, u < v."""
    x = np.asarray(points, np.float32).astype(np.float64)
    n = x.shape[0]
    core2 = core_distances2(points, min_pts)
    if n == 1:
        e = np.empty(0)
        return e.astype(np.int32), e.astype(np.int32), e.astype(np.float64), e.astype(np.float32), e
    # Prim: best[j] = the least (mrd2, min, max) key of an edge from the tree to j
    in_tree = np.zeros(n, bool)
    best_w = np.full(n, np.inf)
    best_a = np.full(n, -1, np.int64)           # tree endpoint of that edge
    edges = []
    cur = 0
    in_tree[0] = True
    ids = np.arange(n)
    for _ in range(n - 1):
        d2 = squared_distances_to(x, cur)
        mr = np.maximum(np.maximum(d2, core2[cur]), core2)
        lo = np.minimum(ids, cur)
        hi = np.maximum(ids, cur)
        blo = np.minimum(ids, best_a)
        bhi = np.maximum(ids, best_a)
        better = (~in_tree) & ((mr < best_w) | ((mr == best_w) & ((lo < blo) | ((lo == blo) & (hi < bhi)))))
        best_w = np.where(better, mr, best_w)
        best_a = np.where(better, cur, best_a)
        # next vertex: least key among the vertices outside the tree
        cand = np.nonzero(~in_tree)[0]
        kw = best_w[cand]
        klo = np.minimum(cand, best_a[cand])
        khi = np.maximum(cand, best_a[cand])
        j = cand[np.lexsort((khi, klo, kw))[0]]
        edges.append((float(best_w[j]), int(min(j, best_a[j])), int(max(j, best_a[j]))))
        in_tree[j] = True
        cur = j
    edges.sort()
    mrd2 = np.array([e[0] for e in edges], np.float64)
    u = np.array([e[1] for e in edges], np.int32)
    v = np.array([e[2] for e in edges], np.int32)
    w64 = np.sqrt(mrd2)
    return u, v, w64, w64.astype(np.float32), mrd2
