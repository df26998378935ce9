"""Independent checkers that pin the oracle (and, later, any output) to what the
paper and plain mathematics fix.  None of these calls the oracle.

* ``brute_force``: connected components at every threshold (the definition of
  the single-linkage hierarchy), O(n^2), for tiny trees.
* ``invariants``: properties every correct dendrogram has (Section 3.1.2
  taxonomy, Section 4.2 count n_alpha = n_leaf - 1, Theorem path_lcda,
  Corollary incident_ancestor).
* ``scipy_merges``: the merge sets of scipy's single linkage on the
  subdominant ultrametric (tie-free inputs only).
"""
from __future__ import annotations

import itertools

import numpy as np


def order_key(w):
    """Ascending (w, id) order as a Python sort (independent of the oracle's qsort)."""
    m = len(w)
    return sorted(range(m), key=lambda i: (float(w[i]), i))


def brute_force(n, u, v, w):
    """Dendrogram by thresholding: after adding the k lightest edges, the parent of
    the k-th edge is the first later edge touching its component; the parent of a
    vertex is the first edge touching it."""
    m = n - 1
    order = order_key(w)
    pos = {e: k for k, e in enumerate(order)}
    ep = [-1] * m
    vp = [-1] * n
    adj = [[] for _ in range(n)]
    for x in range(n):
        first = None
        for e in range(m):
            if u[e] == x or v[e] == x:
                if first is None or pos[e] < pos[first]:
                    first = e
        vp[x] = -1 if first is None else first
    for k, e in enumerate(order):
        adj[u[e]].append(e)
        adj[v[e]].append(e)
        # component of e in the forest of the k+1 lightest edges
        comp = {int(u[e]), int(v[e])}
        stack = list(comp)
        while stack:
            x = stack.pop()
            for f in adj[x]:
                for y in (int(u[f]), int(v[f])):
                    if y not in comp:
                        comp.add(y)
                        stack.append(y)
        for j in range(k + 1, m):
            f = order[j]
            if int(u[f]) in comp or int(v[f]) in comp:
                ep[e] = f
                break
    return np.array(ep, np.int32), np.array(vp, np.int32)


def prufer_trees(n):
    """Every labelled tree on n >= 2 vertices (Cayley: n^(n-2) of them), as edge lists."""
    if n == 2:
        yield [(0, 1)]
        return
    for seq in itertools.product(range(n), repeat=n - 2):
        deg = [1] * n
        for s in seq:
            deg[s] += 1
        edges = []
        for s in seq:
            leaf = min(i for i in range(n) if deg[i] == 1)
            edges.append((leaf, s))
            deg[leaf] -= 1
            deg[s] -= 1
        a = [i for i in range(n) if deg[i] == 1]
        edges.append((a[0], a[1]))
        yield edges


def _key(w, e):
    return (float(w[e]), int(e))


def invariants(n, u, v, w, ep, vp, lcda_pairs=0, seed=0):
    """Assert the structural invariants of a dendrogram; returns the height."""
    m = n - 1
    u = np.asarray(u)
    v = np.asarray(v)
    w = np.asarray(w)
    ep = np.asarray(ep)
    vp = np.asarray(vp)
    assert ep.shape == (m,) and vp.shape == (n,)
    if n == 1:
        assert vp[0] == -1
        return 0
    # exactly one root edge, and it is the heaviest edge
    roots = np.flatnonzero(ep == -1)
    assert len(roots) == 1, f"{len(roots)} roots"
    heaviest = max(range(m), key=lambda e: _key(w, e))
    assert roots[0] == heaviest
    # every parent is an edge and is strictly heavier than its child
    assert np.all((ep >= -1) & (ep < m)) and np.all((vp >= 0) & (vp < m))
    for e in range(m):
        if ep[e] >= 0:
            assert _key(w, ep[e]) > _key(w, e), f"edge {e} parent {ep[e]} not heavier"
    # vertex parent is incident and is the lightest incident edge
    best = {}
    for e in range(m):
        for x in (int(u[e]), int(v[e])):
            if x not in best or _key(w, e) < _key(w, best[x]):
                best[x] = e
    for x in range(n):
        assert vp[x] == best[x], f"vertex {x}: {vp[x]} vs lightest {best[x]}"
    # binary: every edge node has exactly two children
    nchild = np.zeros(m, np.int64)
    nvert = np.zeros(m, np.int64)
    np.add.at(nchild, ep[ep >= 0], 1)
    np.add.at(nchild, vp, 1)
    np.add.at(nvert, vp, 1)
    assert np.all(nchild == 2), "an edge node without exactly two children"
    # Section 4.2: leaf edges (two vertex children) = alpha edges (none) + 1
    assert int((nvert == 2).sum()) == int((nvert == 0).sum()) + 1
    # height (for skewness reporting) and acyclicity
    depth = np.full(m, -1, np.int64)
    for e in range(m):
        path = []
        x = e
        while x >= 0 and depth[x] < 0:
            path.append(x)
            x = ep[x]
            assert len(path) <= m, "cycle in parent pointers"
        d = 0 if x < 0 else depth[x] + 1
        for y in reversed(path):
            depth[y] = d
            d += 1
    height = int(depth.max()) + 1
    # Corollary incident_ancestor: edges sharing a vertex are ancestor-related;
    # checking consecutive incident edges in (w, id) order suffices.
    anc_cache = {}

    def ancestors(e):
        if e not in anc_cache:
            s = set()
            x = e
            while x >= 0:
                s.add(x)
                x = ep[x]
            anc_cache[e] = s
        return anc_cache[e]

    if m <= 4000:
        inc = [[] for _ in range(n)]
        for e in range(m):
            inc[int(u[e])].append(e)
            inc[int(v[e])].append(e)
        for x in range(n):
            es = sorted(inc[x], key=lambda e: _key(w, e))
            for a, b in zip(es, es[1:]):
                assert b in ancestors(a), f"incident edges {a},{b} not ancestor-related"
    # Theorem path_lcda on sampled pairs
    if lcda_pairs and m >= 2:
        rng = np.random.default_rng(seed)
        adj = [[] for _ in range(n)]
        for e in range(m):
            adj[int(u[e])].append((int(v[e]), e))
            adj[int(v[e])].append((int(u[e]), e))
        for _ in range(lcda_pairs):
            a, b = (int(x) for x in rng.integers(0, m, 2))
            # tree path between edge a and edge b: BFS from u[a]
            prev = {int(u[a]): (None, None)}
            q = [int(u[a])]
            for x in q:
                for y, e in adj[x]:
                    if y not in prev:
                        prev[y] = (x, e)
                        q.append(y)
            tgt = int(u[b])
            path_edges = {a, b}
            x = tgt
            while prev[x][0] is not None:
                path_edges.add(prev[x][1])
                x = prev[x][0]
            heaviest_on_path = max(path_edges, key=lambda e: _key(w, e))
            common = ancestors(a) & ancestors(b)
            lcda = min(common, key=lambda e: _key(w, e))
            assert lcda == heaviest_on_path, f"LCDA({a},{b})={lcda}, path max {heaviest_on_path}"
    return height


def scipy_merges(n, u, v, w):
    """Single linkage of the subdominant ultrametric (max weight on the tree path)
    via scipy; returns {edge id: frozenset of child node labels}, where a vertex
    x is ('v', x) and an edge e is ('e', e).  Requires distinct weights."""
    from scipy.cluster.hierarchy import linkage
    from scipy.spatial.distance import squareform

    m = n - 1
    adj = [[] for _ in range(n)]
    for e in range(m):
        adj[int(u[e])].append((int(v[e]), float(w[e])))
        adj[int(v[e])].append((int(u[e]), float(w[e])))
    D = np.zeros((n, n))
    for s in range(n):
        best = {s: 0.0}
        q = [s]
        for x in q:
            for y, wt in adj[x]:
                if y not in best:
                    best[y] = max(best[x], wt)
                    q.append(y)
        for t, d in best.items():
            D[s, t] = d
    Z = linkage(squareform(D, checks=False), method="single")
    by_weight = {float(w[e]): e for e in range(m)}
    assert len(by_weight) == m, "scipy_merges needs distinct weights"
    node = {}
    for x in range(n):
        node[x] = ("v", x)
    out = {}
    for r, row in enumerate(Z):
        e = by_weight[float(row[2])]
        node[n + r] = ("e", e)
        out[e] = frozenset([node[int(row[0])], node[int(row[1])]])
    return out


def children_sets(n, ep, vp):
    out = {}
    for x, p in enumerate(vp):
        if p >= 0:
            out.setdefault(int(p), set()).add(("v", x))
    for e, p in enumerate(ep):
        if p >= 0:
            out.setdefault(int(p), set()).add(("e", e))
    return {k: frozenset(s) for k, s in out.items()}


def brute_flat_clusters(n, u, v, w, mcs):
    """HDBSCAN* flat clusters straight from the definition, for tiny trees.

    No dendrogram: edges are removed from the tree heaviest first (descending
    (w, id)), and each removal splits one connected component, found by a
    search over the remaining edges.  A component owned by a cluster passes it
    on (one part of at least mcs vertices), spawns two new clusters (both parts
    that large) or ends it (neither).  Stabilities are exact rational sums of
    the departure terms count * lambda (each product rounded to fp64, as
    defined) minus size * lambda_birth; the excess-of-mass comparison is exact.
    Returns (labels numbered by smallest vertex id, stabilities as floats in
    label order)."""
    from fractions import Fraction
    m = n - 1
    w32 = np.asarray(w, np.float32)
    lam = [1.0 / float(w32[e]) for e in range(m)]
    order = list(reversed(order_key(w32)))
    alive = set(range(m))

    def component(start):
        seen, stack = {start}, [start]
        while stack:
            x = stack.pop()
            for e in alive:
                a, b = int(u[e]), int(v[e])
                y = b if a == x else a if b == x else None
                if y is not None and y not in seen:
                    seen.add(y)
                    stack.append(y)
        return frozenset(seen)

    # cluster records: points, birth lambda, parent, exact stability
    pts, birth, par, stab, kids = [frozenset(range(n))], [0.0], [None], [Fraction(0)], [[]]
    owner = {frozenset(range(n)): 0}

    def leave(c, count, lm):
        stab[c] += Fraction(float(count) * lm)

    for e in order:
        a, b = int(u[e]), int(v[e])
        K = component(a)
        alive.discard(e)
        K1, K2 = component(a), component(b)
        c = owner.pop(K, None)
        if c is None:
            continue
        lm = lam[e]
        big1, big2 = len(K1) >= mcs, len(K2) >= mcs
        if big1 and big2:
            leave(c, len(K), lm)
            for Kc in (K1, K2):
                pts.append(Kc)
                birth.append(lm)
                par.append(c)
                stab.append(Fraction(0))
                kids.append([])
                kids[c].append(len(pts) - 1)
                owner[Kc] = len(pts) - 1
        elif big1 or big2:
            leave(c, len(K2) if big1 else len(K1), lm)
            owner[K1 if big1 else K2] = c
        else:
            leave(c, len(K), lm)
    for c in range(1, len(pts)):
        stab[c] -= Fraction(float(len(pts[c])) * birth[c])

    # excess of mass (children were appended after their parents)
    value, sel = {}, {}
    for c in range(len(pts) - 1, 0, -1):
        if kids[c]:
            cs = sum(value[k] for k in kids[c])
            sel[c] = stab[c] >= cs
            value[c] = stab[c] if sel[c] else cs
        else:
            sel[c], value[c] = True, stab[c]
    chosen = []
    for c in range(1, len(pts)):
        a, ok = par[c], sel[c]
        while ok and a not in (None, 0):
            ok = not sel[a]
            a = par[a]
        if ok:
            chosen.append(c)
    lab = np.full(n, -1, np.int32)
    for c in chosen:
        for x in pts[c]:
            lab[x] = c
    out, names, st = np.full(n, -1, np.int32), {}, []
    for x in range(n):
        if lab[x] >= 0:
            if lab[x] not in names:
                names[lab[x]] = len(names)
                st.append(float(stab[lab[x]]))
            out[x] = names[lab[x]]
    return out, np.array(st, np.float64)
