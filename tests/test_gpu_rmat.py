"""Checks on the R-MAT workload: scale 22, edge factor 24, (a, b, c) = (0.57,
0.19, 0.19), symmetrised and deduplicated (about 95M edges), plus 50 cliques
of 20..60 vertices planted on disjoint random vertex sets.

Its degeneracy is 1318 and its tree cannot be walked whole, neither for all k
nor truncated at k = 8: a single root of out-degree above 512 already keeps
the oracle busy for minutes.  So parity at this size is the peel order of
every vertex and the degeneracy, and the all-k and truncated counts, tree
sizes and clique numbers of a seeded sample of roots in four out-degree
strata (up to 512, so heavy roots with up to 8 words per row are included),
against the oracle on the same roots.  Whole-graph per-edge counts are not
checked here for the same reason; per-edge parity is covered on smaller
graphs.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_06784_amd import graphgen as gg
from paper_2001_06784_amd import pivoter as P

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rmat22():
    _say("[rmat22] generating")
    g = gg.rmat_web()
    _say(f"[rmat22] n={g.n} m={g.m}")
    ctx = P.pv_init(0)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    alpha = P.pv_graph_orient(h)
    sub = P.pv_graph_export_order(h)
    _say(f"[rmat22] oriented: alpha={alpha}")
    yield g, h, alpha, sub
    P.pv_graph_free(h)
    P.pv_fini(ctx)


def _sample(g, sub):
    od = O.out_degrees(g, sub)
    rng = np.random.default_rng(2022)
    parts = []
    for lo, hi, cnt in [(0, 64, 2000), (64, 128, 40), (128, 256, 10), (256, 512, 5)]:
        pool = np.nonzero((od > lo) & (od <= hi))[0]
        parts.append(rng.choice(pool, min(cnt, len(pool)), replace=False))
    parts.append(np.nonzero(od == 0)[0][:5])
    return np.concatenate(parts).astype(np.int32), od


def test_rmat22_peel_order(rmat22):
    g, h, alpha, sub = rmat22
    pe = O.peel(g)
    assert np.array_equal(sub, pe.sub), "peel order differs"
    assert alpha == pe.alpha and alpha > 1024


@pytest.mark.parametrize("kmax", [0, 8])
def test_rmat22_sampled_roots(rmat22, kmax):
    g, h, alpha, sub = rmat22
    roots, od = _sample(g, sub)
    _say(f"[rmat22] {len(roots)} sampled roots, largest out-degree {int(od[roots].max())}, kmax={kmax}")
    got = P.pv_count_roots(h, roots, k_max=kmax)
    ref = O.count(g, key=sub, roots=roots, kmax=kmax)
    _say(f"[rmat22] nodes={ref.stats['nodes']} leaves={ref.stats['leaves']} omega={ref.omega}")
    top = len(ref.glob)
    assert got.overflow == [k for k in range(top) if ref.glob_ovf[k]]
    assert got.counts[1:top] == ref.glob[1:]
    assert all(c == 0 for c in got.counts[top:])
    assert got.omega == (min(ref.omega, kmax) if kmax else ref.omega)
    if not kmax:
        assert got.stats["leaves"] == ref.stats["leaves"]
        assert got.stats["nodes"] == ref.stats["nodes"]
