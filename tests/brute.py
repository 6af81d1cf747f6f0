"""Independent ground truth for tiny and small graphs (test helpers).

Nothing here uses pivoting, orientation or the Succinct Clique Tree: the
brute force checks every vertex subset, and the enumerator is the simple
backtracking clique lister (Sec. 2: recurse on N(s) intersected with S for
every s, with each clique produced once by only extending with larger ids).
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np


def adjacency_sets(g):
    return [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]


def edge_index(g):
    a, b = g.edges()
    return {(int(x), int(y)): i for i, (x, y) in enumerate(zip(a, b))}


def brute_counts(g):
    """All cliques by subset enumeration (n <= ~16).  Returns (C, cv, ce):
    C[k], cv[v][k], ce[eid][k] as Python ints, k = 0..n."""
    n = g.n
    adj = adjacency_sets(g)
    eidx = edge_index(g)
    C = [0] * (n + 2)
    cv = [[0] * (n + 2) for _ in range(n)]
    ce = [[0] * (n + 2) for _ in range(len(eidx))]
    for mask in range(1 << n):
        vs = [v for v in range(n) if (mask >> v) & 1]
        ok = all(b in adj[a] for a, b in itertools.combinations(vs, 2))
        if not ok:
            continue
        k = len(vs)
        C[k] += 1
        for v in vs:
            cv[v][k] += 1
        for a, b in itertools.combinations(vs, 2):
            ce[eidx[(a, b)]][k] += 1
    return C, cv, ce


def enumerate_cliques(g, kmax=None):
    """Simple backtracking lister: every clique once, as increasing tuples."""
    adj = adjacency_sets(g)
    up = [sorted(u for u in adj[v] if u > v) for v in range(g.n)]
    out = []

    def extend(clique, cand):
        out.append(tuple(clique))
        if kmax is not None and len(clique) >= kmax:
            return
        for i, s in enumerate(cand):
            extend(clique + [s], [t for t in cand[i + 1:] if t in adj[s]])

    for v in range(g.n):
        extend([v], up[v])
    return out


def enum_counts(g, kmax=None):
    cl = enumerate_cliques(g, kmax)
    top = max((len(c) for c in cl), default=0)
    C = [0] * (top + 2)
    C[0] = 1
    for c in cl:
        C[len(c)] += 1
    return C, cl


def elementary_symmetric(parts, k):
    """e_k(a_1, ..., a_r)."""
    e = [1] + [0] * k
    for a in parts:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * a
    return e[k]


def matula_beck_degeneracy(g):
    """Degeneracy by repeatedly deleting one minimum-degree vertex."""
    adj = adjacency_sets(g)
    deg = {v: len(adj[v]) for v in range(g.n)}
    alive = set(range(g.n))
    best = 0
    while alive:
        v = min(alive, key=lambda x: (deg[x], x))
        best = max(best, deg[v])
        alive.remove(v)
        for u in adj[v]:
            if u in alive:
                deg[u] -= 1
    return best


def triangles_by_matrix(g):
    a = np.zeros((g.n, g.n), dtype=np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a[src, g.col] = 1
    return int(np.trace(a @ a @ a) // 6)
