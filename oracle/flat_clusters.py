"""CPU oracle for HDBSCAN* flat clusters taken from the single-linkage
dendrogram of an MST.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
loads it, and the two share no code.

The paper (Section "HDBSCAN* Performance") names flat-cluster extraction as
the optional step after the dendrogram and takes the method from Campello et
al. (2015), its HDBSCAN* reference.  What is computed here, for a minimum
cluster size mcs >= 2:

* Density level of an edge: lambda(e) = 1 / w(e) in fp64 (w = +inf gives 0).
  Every weight must be > 0.
* size(x) = 1 for a vertex; size(e) = number of vertices below edge node e.
* Walking the dendrogram from the root down, an edge node e splits its
  cluster.  If both of its children hold at least mcs vertices, the split is
  true: both children are born as new clusters at lambda(e), and the cluster
  of e ends there.  If exactly one child is that large, the vertices of the
  small child leave the cluster at lambda(e), and the cluster goes on into the
  large child.  If neither is, all size(e) vertices leave at lambda(e), and
  the cluster ends.  The whole tree is the root cluster, born at lambda 0.
* Stability of a cluster C born at lambda_b: the sum over its vertices of
  (lambda at which the vertex leaves C) - lambda_b.  Per departure event that
  is count * lambda; the birth term is size(C) * lambda_b.  Each product is
  one fp64 multiplication; the sum is exactly rounded (math.fsum).
* Excess-of-mass selection, bottom up over the cluster tree: a cluster whose
  stability is at least the summed value of its two children is selected
  (its value is its stability), otherwise its value is that sum.  The root
  is never selected.  The chosen clusters are the selected ones with no
  selected ancestor.
* A vertex gets the label of the chosen cluster it belongs to, else -1
  (noise).  Labels are numbered in order of their smallest vertex id.

Every step runs on the dendrogram from ``oracle.dendrogram`` with plain
loops over edges in rank order (children always precede their parents).
"""
from __future__ import annotations

import math

import numpy as np

from . import dendrogram, edge_order

ROOT = -2   # cluster id of the root cluster (clusters are named by birth edge)


def _check(n, w, mcs):
    if n < 1 or mcs < 2:
        raise ValueError("need n >= 1 and min_cluster_size >= 2")
    w = np.asarray(w, np.float32)
    if w.size and not np.all(w > 0):
        raise ValueError("flat clusters need every weight > 0")


def flat_clusters(n, u, v, w, mcs, *, return_info=False):
    """(labels int32[n], stability float64[k] of the chosen clusters in label
    order[, info]).  ``info`` holds what the parity tests need to tell safe
    selection decisions from near-ties (see ``decisions``)."""
    _check(n, w, mcs)
    n = int(n)
    m = n - 1
    w = np.ascontiguousarray(w, np.float32)
    if n == 1:
        lab = np.full(1, -1, np.int32)
        st = np.zeros(0, np.float64)
        return (lab, st, {"decisions": []}) if return_info else (lab, st)
    ep, vp = dendrogram(n, u, v, w)
    order = edge_order(w)                       # ascending (w, id)
    lam = 1.0 / w.astype(np.float64)            # +inf weight -> 0.0

    # sizes: vertices, then edges in ascending rank (children come first)
    size = np.zeros(m, np.int64)
    np.add.at(size, vp, 1)
    epl = ep.tolist()
    sz = size.tolist()
    for e in order.tolist():
        p = epl[e]
        if p >= 0:
            sz[p] += sz[e]
    size = np.array(sz, np.int64)

    # children of each edge node that hold >= mcs vertices (vertices never do)
    big = [0] * m
    bigmax = [0] * m
    for e in range(m):
        p = epl[e]
        if p >= 0 and sz[e] >= mcs:
            big[p] += 1
            bigmax[p] = max(bigmax[p], sz[e])

    # cluster of every edge node, top down (descending rank): its own birth or
    # its parent's cluster
    T = [0] * m
    for e in reversed(order.tolist()):
        p = epl[e]
        if p < 0:
            T[e] = ROOT
        elif sz[e] >= mcs and big[p] == 2:
            T[e] = e
        else:
            T[e] = T[p]

    # departures: every edge node of a cluster's region (size >= mcs)
    terms: dict[int, list[float]] = {}
    births = []
    for e in range(m):
        if sz[e] < mcs:
            continue
        if big[e] == 1:
            d = sz[e] - bigmax[e]
        else:
            d = sz[e]
        terms.setdefault(T[e], []).append(float(d) * float(lam[e]))
        if T[e] == e:
            births.append(e)
    clusters = {}
    for c in births:
        tl = terms.get(c, [])
        tl.append(-(float(sz[c]) * float(lam[epl[c]])))
        clusters[c] = tl
    stab = {c: math.fsum(tl) for c, tl in clusters.items()}
    abs_sum = {c: math.fsum(abs(t) for t in tl) for c, tl in clusters.items()}
    nterms = {c: len(tl) for c, tl in clusters.items()}

    # cluster tree: parent cluster of a birth is the cluster of its parent node
    parent = {c: T[epl[c]] for c in births}
    children: dict[int, list[int]] = {}
    for c in births:
        children.setdefault(parent[c], []).append(c)

    # excess of mass, bottom up: children are born below their parent, so
    # ascending rank of the birth edge visits children first
    rank = np.empty(m, np.int64)
    rank[order] = np.arange(m)
    value, sel, decisions = {}, {}, []
    u53 = 2.0 ** -53
    err = {}
    for c in sorted(births, key=lambda e: rank[e]):
        k = nterms[c]
        e_stab = (k * u53 / (1 - k * u53)) * abs_sum[c]
        ch = children.get(c, [])
        if not ch:
            value[c], sel[c], err[c] = stab[c], True, e_stab
            continue
        assert len(ch) == 2
        cs = value[ch[0]] + value[ch[1]]
        e_cs = err[ch[0]] + err[ch[1]] + u53 * abs(cs)
        sel[c] = stab[c] >= cs
        value[c] = stab[c] if sel[c] else cs
        err[c] = max(e_stab, e_cs)
        decisions.append((c, stab[c], cs, e_stab + e_cs))

    # chosen: selected with no selected ancestor (top down, descending rank)
    chosen_of = {ROOT: None}
    anc_sel = {ROOT: False}
    for c in sorted(births, key=lambda e: -rank[e]):
        p = parent[c]
        a = anc_sel[p]
        chosen_of[c] = c if (sel[c] and not a) else chosen_of[p]
        anc_sel[c] = a or sel[c]

    # labels: a vertex belongs to the cluster of its parent edge node (vertices
    # are never born: mcs >= 2), numbered by smallest vertex id
    lab = np.full(n, -1, np.int32)
    first: dict[int, int] = {}
    out_stab = []
    vpl = vp.tolist()
    for x in range(n):
        c = chosen_of[T[vpl[x]]]
        if c is None:
            continue
        if c not in first:
            first[c] = len(first)
            out_stab.append(stab[c])
        lab[x] = first[c]
    st = np.array(out_stab, np.float64)
    if not return_info:
        return lab, st
    info = {"decisions": decisions, "stability": stab, "abs_sum": abs_sum, "nterms": nterms,
            "chosen": [c for c in first], "size": size}
    return lab, st, info


def decisions_safe(info, factor=2.0) -> bool:
    """True when every selection decision is farther from a tie than the
    summation error bound (times ``factor``): then any summation order of
    the same fp64 terms takes the same decisions."""
    return all(abs(s - cs) > factor * bound for _, s, cs, bound in info["decisions"])
