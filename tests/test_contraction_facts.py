"""Two facts about tree contraction (paper, Sec. 3.2 and Sec. 4.2) that the
GPU path relies on, checked on a plain Python model of the levels, on random
trees with heavy weight ties:

  1. the leaf edge of every non-alpha component is lighter than every alpha
     edge incident to that component, so in the expansion (Sec. 3.3.2) it
     always belongs to its own supervertex's chain (the level kernels write
     its chain directly and the walk skips it);
  2. a level of a forest has at most half as many vertices as the level
     before (one per leaf edge), which bounds the chain keys of the levels
     still to come.

The model shares nothing with the library: per level it takes every
vertex's lightest incident edge, marks edges owned by neither endpoint as
alpha and by both as leaf edges, joins the non-alpha edges into components
and contracts each component to one vertex."""
import numpy as np
import pytest

import gen


def contract(n, edges):
    """One level: edges are (u, v, rank).  Returns the next level's
    (n, edges) and checks both facts on the way."""
    light = [None] * n
    for u, v, r in edges:
        for x in (u, v):
            if light[x] is None or r < light[x]:
                light[x] = r
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    alpha, leaves = [], []
    for u, v, r in edges:
        own_u, own_v = light[u] == r, light[v] == r
        if not own_u and not own_v:
            alpha.append((u, v, r))
            continue
        if own_u and own_v:
            leaves.append((u, v, r))
        parent[find(u)] = find(v)
    leaf_of = {}
    for u, v, r in leaves:
        c = find(u)
        assert c not in leaf_of, "one leaf edge per component"
        leaf_of[c] = r
    lightest_alpha = {}
    for u, v, r in alpha:
        for x in (u, v):
            c = find(x)
            lightest_alpha[c] = min(lightest_alpha.get(c, r), r)
    for c, r_alpha in lightest_alpha.items():
        assert leaf_of[c] < r_alpha, "fact 1: the leaf edge is lighter than every alpha edge at its component"
    label = {c: k for k, c in enumerate(sorted(leaf_of))}
    n_next = len(label)
    assert 2 * n_next <= n, "fact 2: at most half the vertices"
    nxt = [(label[find(u)], label[find(v)], r) for u, v, r in alpha]
    return n_next, nxt


def ranks(w):
    order = np.lexsort((np.arange(len(w)), w))
    r = np.empty(len(w), dtype=np.int64)
    r[order] = np.arange(len(w))
    return r


@pytest.mark.parametrize("seed", range(40))
def test_facts_on_random_trees(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    kind = seed % 4
    if kind == 0:
        t = gen.rrt(n, seed)
    elif kind == 1:
        t = gen.shuffled(gen.pref_attach(n, seed), seed)
    elif kind == 2:
        t = gen.caterpillar(max(n, 3), None, 1e-3, seed)
    else:
        t = gen.star(n, seed)
    w = t.w.copy()
    if seed % 3 == 0:
        w = np.floor(w * 4).astype(np.float32)     # heavy ties: order falls to the edge id
    r = ranks(w)
    level_n, edges = t.n, [(int(a), int(b), int(c)) for a, b, c in zip(t.u, t.v, r)]
    levels = 0
    while edges:
        level_n, edges = contract(level_n, edges)
        levels += 1
    assert levels <= int(np.ceil(np.log2(t.n))) + 1


def test_facts_on_a_forest():
    """Several trees side by side (the batched mode): fact 2 holds for the
    whole level, since every component has at most (m + 1) / 2 leaf edges."""
    trees = [gen.rrt(5 + 17 * k, k) for k in range(12)] + [gen.star(30, 3)]
    n, edges, w = 0, [], []
    for t in trees:
        edges += [(int(a) + n, int(b) + n) for a, b in zip(t.u, t.v)]
        w += list(t.w)
        n += t.n
    r = ranks(np.asarray(w, dtype=np.float32))
    level_n, es = n, [(a, b, int(c)) for (a, b), c in zip(edges, r)]
    while es:
        level_n, es = contract(level_n, es)
