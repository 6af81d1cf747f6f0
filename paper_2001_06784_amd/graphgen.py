"""Seeded synthetic graph generators shared by the tests, the benchmark and the
oracle-side checks.

This module holds no step of the counting method: it only draws edge lists and
packs them into a simple, symmetric, sorted int32 CSR (the input form of the
problem statement, Sec. 1.1: an undirected simple graph).  Every generator
takes an explicit seed and uses numpy's PCG64, so the same call always yields
the same graph on every machine.

Shapes follow the workloads of the experiments (Sec. 6): the paper measures
heavy-tailed social and web networks, which are stood in for here by
Chung-Lu power-law graphs and R-MAT graphs; the small families (complete,
complete multipartite, Moon-Moser, cycles, ...) have closed-form clique
counts and are used as test pins.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    """Simple undirected graph as a symmetric CSR with sorted rows.

    row_ptr: int32[n+1], col: int32[2m].  Row v lists the neighbours of v in
    increasing id order; no self loops, no duplicates, (u,v) present iff (v,u)
    present.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def m(self) -> int:
        return int(self.col.shape[0] // 2)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def edges(self) -> tuple[np.ndarray, np.ndarray]:
        """Undirected edges (u < v) in lexicographic order."""
        src = np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr))
        keep = src < self.col
        return src[keep], self.col[keep]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def from_edges(n: int, u, v) -> Graph:
    """Symmetrise, drop self loops and duplicates, sort; return CSR."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.size:
        if u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n:
            raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    both = np.concatenate([key, b * n + a])
    both.sort()
    src = both // n
    dst = both % n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32))


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    a, b = g.edges()
    return from_edges(g.n, perm[a], perm[b])


# ---------------------------------------------------------------- families

def empty(n: int) -> Graph:
    return from_edges(n, [], [])


def complete(n: int) -> Graph:
    iu = np.triu_indices(n, 1)
    return from_edges(n, iu[0], iu[1])


def complete_multipartite(parts) -> Graph:
    """K_{a_1,...,a_r}: vertices in different parts are adjacent."""
    parts = [int(a) for a in parts]
    n = sum(parts)
    label = np.repeat(np.arange(len(parts)), parts)
    iu = np.triu_indices(n, 1)
    keep = label[iu[0]] != label[iu[1]]
    return from_edges(n, iu[0][keep], iu[1][keep])


def moon_moser(r: int) -> Graph:
    """Complete r-partite graph with parts of size 3 (3^r maximal cliques)."""
    return complete_multipartite([3] * r)


def cycle(n: int) -> Graph:
    a = np.arange(n)
    return from_edges(n, a, (a + 1) % n)


def path(n: int) -> Graph:
    a = np.arange(max(n - 1, 0))
    return from_edges(n, a, a + 1)


def star(n: int) -> Graph:
    return from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))


def gnp(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n,p): each pair i<j independently with probability p."""
    rng = _rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p
    return from_edges(n, iu[0][keep], iu[1][keep])


def disjoint_union(g: Graph, h: Graph) -> Graph:
    a1, b1 = g.edges()
    a2, b2 = h.edges()
    return from_edges(g.n + h.n, np.concatenate([a1, a2 + g.n]),
                      np.concatenate([b1, b2 + g.n]))


def join(g: Graph, h: Graph) -> Graph:
    """Disjoint union plus every edge between the two vertex sets."""
    a1, b1 = g.edges()
    a2, b2 = h.edges()
    x, y = np.meshgrid(np.arange(g.n), np.arange(h.n) + g.n, indexing="ij")
    return from_edges(g.n + h.n,
                      np.concatenate([a1, a2 + g.n, x.ravel()]),
                      np.concatenate([b1, b2 + g.n, y.ravel()]))


def plant_cliques(g: Graph, sizes, seed: int) -> Graph:
    """Add cliques on disjoint, uniformly chosen vertex sets."""
    sizes = [int(s) for s in sizes]
    if sum(sizes) > g.n:
        raise ValueError("planted cliques do not fit")
    rng = _rng(seed)
    verts = rng.permutation(g.n)[: sum(sizes)]
    a, b = g.edges()
    ea, eb = [a.astype(np.int64)], [b.astype(np.int64)]
    off = 0
    for s in sizes:
        vs = verts[off: off + s]
        off += s
        iu = np.triu_indices(s, 1)
        ea.append(vs[iu[0]])
        eb.append(vs[iu[1]])
    return from_edges(g.n, np.concatenate(ea), np.concatenate(eb))


# ---------------------------------------------------- heavy-tailed workloads

def chung_lu_weights(n: int, avg_deg: float, gamma: float, max_deg: float) -> np.ndarray:
    """Power-law expected degrees w_i ~ c * (i+1)^(-1/(gamma-1)), capped at
    max_deg, with c chosen so that mean(w) = avg_deg."""
    beta = 1.0 / (gamma - 1.0)
    base = np.arange(1, n + 1, dtype=np.float64) ** (-beta)
    target = min(float(avg_deg), float(max_deg))
    lo, hi = 0.0, 1.0
    while np.minimum(hi * base, max_deg).mean() < target:
        hi *= 2.0
    for _ in range(200):
        c = 0.5 * (lo + hi)
        if np.minimum(c * base, max_deg).mean() < target:
            lo = c
        else:
            hi = c
    return np.minimum(hi * base, max_deg)


def chung_lu(n: int, avg_deg: float, gamma: float, max_deg: float, seed: int,
             shuffle: bool = True) -> Graph:
    """Chung-Lu graph by endpoint sampling: n*avg_deg/2 pairs with both ends
    drawn i.i.d. proportional to the weights; loops and duplicates dropped.
    Vertex ids are randomly permuted (seeded) so that hubs are spread over the
    id range."""
    rng = _rng(seed)
    w = chung_lu_weights(n, avg_deg, gamma, max_deg)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    npairs = int(round(n * avg_deg / 2.0))
    u = np.searchsorted(cdf, rng.random(npairs), side="right")
    v = np.searchsorted(cdf, rng.random(npairs), side="right")
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    if shuffle:
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
    return from_edges(n, u, v)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> Graph:
    """R-MAT: edge_factor * 2^scale samples, each choosing one quadrant per bit
    with probabilities (a, b, c, 1-a-b-c); symmetrised, loops and duplicates
    dropped."""
    rng = _rng(seed)
    n = 1 << scale
    ne = edge_factor * n
    u = np.zeros(ne, dtype=np.int64)
    v = np.zeros(ne, dtype=np.int64)
    chunk = 1 << 22
    for s in range(0, ne, chunk):
        e = min(ne, s + chunk)
        uu = np.zeros(e - s, dtype=np.int64)
        vv = np.zeros(e - s, dtype=np.int64)
        for bit in range(scale):
            r = rng.random(e - s)
            right = (r >= a) & (r < a + b) | (r >= a + b + c)
            down = r >= a + b
            uu |= down.astype(np.int64) << bit
            vv |= right.astype(np.int64) << bit
        u[s:e] = uu
        v[s:e] = vv
    return from_edges(n, u, v)


# ----------------------------------------------------- benchmark workloads

def er_planted(n: int = 2000, p: float = 0.01, clique_sizes=(12, 12, 12),
               seed: int = 1, plant_seed: int = 2) -> Graph:
    """G(n,p) plus cliques planted on disjoint random vertex sets."""
    return plant_cliques(gnp(n, p, seed), clique_sizes, plant_seed)


def chung_lu_social(n: int = 1_000_000, avg_deg: float = 20.0, gamma: float = 2.3,
                    max_deg: float = 20_000.0, seed: int = 1) -> Graph:
    """Heavy-tailed stand-in for the paper's social networks."""
    return chung_lu(n, avg_deg, gamma, max_deg, seed)


def rmat_web(scale: int = 22, edge_factor: int = 24, a: float = 0.57, b: float = 0.19, c: float = 0.19,
             seed: int = 1, cliques: int = 50, clique_lo: int = 20, clique_hi: int = 60,
             plant_seed: int = 2) -> Graph:
    """Heavy-tailed web-like stand-in: R-MAT plus `cliques` cliques whose sizes
    are uniform on {clique_lo..clique_hi}, planted on disjoint random vertex
    sets (sizes and sets drawn from plant_seed)."""
    g = rmat(scale, edge_factor, a, b, c, seed)
    sizes = _rng(plant_seed).integers(clique_lo, clique_hi + 1, cliques)
    return plant_cliques(g, sizes, plant_seed + 1)


def batch_graph_specs(count: int = 4096, n_lo: int = 50, n_hi: int = 5000,
                      deg_lo: float = 8.0, deg_hi: float = 40.0, seed: int = 1000):
    """(n, avg_deg, seed) of each member of a batch of small Chung-Lu graphs:
    n log-uniform in [n_lo, n_hi], average degree uniform in [deg_lo, deg_hi]
    (capped at n-1)."""
    rng = _rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    ds = rng.uniform(deg_lo, deg_hi, count)
    out = []
    for i in range(count):
        n = int(ns[i])
        d = float(min(ds[i], n - 1))
        out.append((n, d, seed + i))
    return out


def batch_graphs(count: int = 4096, gamma: float = 2.5, **kw) -> list[Graph]:
    return [chung_lu(n, d, gamma, n - 1, s) for (n, d, s) in batch_graph_specs(count, **kw)]


def serve_pool_specs(count: int = 256, m_lo: float = 1e3, m_hi: float = 2e6,
                     deg_lo: float = 8.0, deg_hi: float = 40.0, seed: int = 3):
    """(n, avg_deg, seed) of a pool of Chung-Lu graphs with edge counts
    log-uniform in [m_lo, m_hi]."""
    rng = _rng(seed)
    ms = np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), count))
    ds = rng.uniform(deg_lo, deg_hi, count)
    out = []
    for i in range(count):
        n = max(int(round(2.0 * ms[i] / ds[i])), 16)
        out.append((n, float(min(ds[i], n - 1)), seed * 100000 + i))
    return out


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Open-loop arrival times (seconds) of a Poisson stream."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, int(rate * duration * 2) + 16)
    t = np.cumsum(gaps)
    return t[t < duration]
