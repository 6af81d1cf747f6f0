"""The multi-word tier at nine and more 64-bit words per set (|N+(v)| > 512),
checked against closed forms that hold at any size.

Complete graphs K_n: C_k = C(n, k); every root child N+(v) is a clique
walked as one pivot chain, so the tree has n leaves and n(n+1)/2 nodes, its
pivot work is sum over d < n of (n - d) d ceil(d/64), and its child work
(one pivot child per node of size j > 0) sum over j < n of (n - j) ceil(j/64).  Per vertex,
c_k(v) = C(n-1, k-1); per edge, c_k(e) = C(n-2, k-2).  Complete multipartite
graphs: C_k = e_k(part sizes) (one vertex from each of k distinct parts).
Counts reach thousands of bits, so the wide read-off is used.
"""
import sys
from math import comb

import numpy as np
import pytest

from paper_2001_06784_amd import graphgen as gg
from paper_2001_06784_amd import pivoter as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.pv_init(0)
    yield c
    P.pv_fini(c)


def _elementary_symmetric(parts):
    e = [1]
    for a in parts:
        e = [x + (a * e[i - 1] if i else 0) for i, x in enumerate(e + [0])]
    return e


def _words(d):
    return (d + 63) // 64


@pytest.mark.parametrize("n", [600, 1100, 1320])
def test_complete_graph_many_words(ctx, n):
    _say(f"[multiword] K_{n}: {_words(n - 1)} words per set")
    g = gg.complete(n)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        res = P.pv_count_global_wide(h, cap=n + 2, limbs=n // 64 + 2)
    finally:
        P.pv_graph_free(h)
    assert _words(res.stats["alpha"]) >= 9
    assert res.stats["alpha"] == n - 1
    assert res.omega == n and not res.overflow
    assert res.counts[: n + 2] == [comb(n, k) for k in range(n + 2)]
    assert res.stats["leaves"] == n
    assert res.stats["nodes"] == n * (n + 1) // 2
    assert res.stats["work"] == sum((n - d) * d * _words(d) for d in range(n))
    # a node of size j has one child (its pivot child) of j words' formation
    assert res.stats["child_work"] == sum((n - j) * _words(j) for j in range(1, n))
    # root v_i's one leaf has h = 1, p = n - 1 - i
    assert res.stats["leaf_hp"] == n * (n + 1) // 2
    assert res.stats["leaf_pp"] == n * (n + 1) // 2


def test_complete_graph_u128_read_off_truncated(ctx):
    # truncated at k_max = 12 every C(1320, k), k <= 12, fits 128 bits
    g = gg.complete(1320)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        res = P.pv_count_global(h, k_max=12)
    finally:
        P.pv_graph_free(h)
    assert res.counts[:14] == [comb(1320, k) for k in range(13)] + [0]
    assert res.omega == 12


def test_multipartite_with_700_singleton_parts(ctx):
    parts = [1] * 700 + [2, 3, 3]
    g = gg.complete_multipartite(parts)
    want = _elementary_symmetric(parts)
    _say(f"[multiword] complete multipartite, {len(parts)} parts, n={g.n}")
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        res = P.pv_count_global_wide(h, cap=len(parts) + 2, limbs=13)
    finally:
        P.pv_graph_free(h)
    assert _words(res.stats["alpha"]) >= 9
    assert res.omega == len(parts) and not res.overflow
    assert res.counts[: len(want)] == want
    assert res.counts[len(want)] == 0
    # every maximal clique (one vertex of each part: 2 * 3 * 3 of them) is
    # H + P of a leaf of its own (Thm. scr: it is H + Q for one leaf, and
    # H + P is a clique containing it)
    assert res.stats["leaves"] >= 18


def test_complete_graph_per_vertex_many_words(ctx):
    n = 600
    g = gg.complete(n)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, 1, 8)
    finally:
        P.pv_graph_free(h)
    assert ovf == 0
    for k in range(1, 9):
        want = comb(n - 1, k - 1)
        col = out[:, k - 1]
        assert (col[:, 0] == np.uint64(want & (2 ** 64 - 1))).all(), k
        assert (col[:, 1] == np.uint64(want >> 64)).all(), k


def test_complete_graph_per_edge_many_words(ctx):
    n = 600
    g = gg.complete(n)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        out, ovf, st = P.pv_count_local(h, P.PV_EDGE, 2, 6)
    finally:
        P.pv_graph_free(h)
    assert ovf == 0 and out.shape[0] == n * (n - 1) // 2
    for k in range(2, 7):
        want = comb(n - 2, k - 2)
        col = out[:, k - 2]
        assert (col[:, 0] == np.uint64(want)).all() and (col[:, 1] == 0).all(), k
