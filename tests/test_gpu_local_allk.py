"""Per-vertex and per-edge counts for every k (Alg. 2's vertex and pair
steps over the whole range of k) on graphs whose degeneracy passes 67, where
the binomials the read-off needs pass 64 bits.  Parity with the oracle,
element by element, and closed forms of complete graphs up to and past
2^128.
"""
import sys
from math import comb

import numpy as np
import pytest

from oracle import oracle as O
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


def _local(ctx, g, kind, klo, khi):
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        alpha = P.pv_graph_orient(h)
        out, ovf, st = P.pv_count_local(h, kind, klo, khi)
    finally:
        P.pv_graph_free(h)
    return out, ovf, alpha


def _planted():
    return gg.plant_cliques(gg.gnp(600, 0.05, 71), [75, 40], 72)


def test_per_vertex_every_k_high_degeneracy(ctx):
    g = _planted()
    ref = O.count(g, vertex=(1, 76))
    out, ovf, alpha = _local(ctx, g, P.PV_VERTEX, 1, 76)
    _say(f"[allk] per vertex k=1..76: alpha={alpha} omega={ref.omega}")
    assert alpha > 67 and ref.omega == 75
    assert comb(74, 37) > 2 ** 64  # the read-off needs binomials past 64 bits
    assert ovf == 0 and not ref.vertex_ovf.any()
    assert np.array_equal(out, ref.vertex)


def test_per_edge_every_k_high_degeneracy(ctx):
    g = _planted()
    ref = O.count(g, edge=(2, 76))
    out, ovf, alpha = _local(ctx, g, P.PV_EDGE, 2, 76)
    assert alpha > 67 and ovf == 0 and not ref.edge_ovf.any()
    assert np.array_equal(out, ref.edge)


def test_complete_131_every_k(ctx):
    # C(130, k-1) < 2^128 for every k: all exact, many past 2^64
    n = 131
    out, ovf, _ = _local(ctx, gg.complete(n), P.PV_VERTEX, 1, n)
    assert ovf == 0
    for k in range(1, n + 1):
        want = comb(n - 1, k - 1)
        assert (out[:, k - 1, 0] == np.uint64(want & (2 ** 64 - 1))).all(), k
        assert (out[:, k - 1, 1] == np.uint64(want >> 64)).all(), k


def test_complete_140_overflow_is_flagged(ctx):
    # c_k(v) = C(139, k-1) passes 2^128 for k - 1 in the middle: flagged,
    # while every column below 2^128 is still exact
    n = 140
    out, ovf, _ = _local(ctx, gg.complete(n), P.PV_VERTEX, 1, n)
    assert ovf != 0
    exact = [k for k in range(1, n + 1) if comb(n - 1, k - 1) < 2 ** 128]
    assert len(exact) < n
    for k in exact:
        want = comb(n - 1, k - 1)
        assert (out[:, k - 1, 0] == np.uint64(want & (2 ** 64 - 1))).all(), k
        assert (out[:, k - 1, 1] == np.uint64(want >> 64)).all(), k


def test_per_edge_complete_140_small_k(ctx):
    # k <= 8 on K_140: C(138, k-2) fits, and the rows of 132+ pivots are
    # checked for overflow without a false flag
    out, ovf, _ = _local(ctx, gg.complete(140), P.PV_EDGE, 2, 8)
    assert ovf == 0
    for k in range(2, 9):
        assert (out[:, k - 2, 0] == np.uint64(comb(138, k - 2))).all() and (out[:, k - 2, 1] == 0).all()
