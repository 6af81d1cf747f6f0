"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Everything here is integer work, so the bar is bit-exact equality: the peel
order, the global counts C_k (exact u128, with identical overflow flags), the
clique number, the SCT's node and leaf counts (the GPU follows the same pivot
and child-order rules, so it builds the same tree), and per-vertex counts.
"""
import os
import sys

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


class Loaded:
    def __init__(self, ctx, g):
        self.h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)

    def __enter__(self):
        return self.h

    def __exit__(self, *exc):
        P.pv_graph_free(self.h)


def check_global(ctx, g, name, kmax=0, check_order=True):
    _say(f"[parity] {name}: n={g.n} m={g.m} kmax={kmax}")
    with Loaded(ctx, g) as h:
        res = P.pv_count_global(h, kmax)
        sub = P.pv_graph_export_order(h)
    if check_order:
        pe = O.peel(g)
        assert np.array_equal(sub, pe.sub), "peel order differs"
    ref = O.count(g, key=sub, kmax=kmax, hist_dim=res.stats["alpha"] + 2)
    assert ref.stats["hist_out"] == 0
    top = len(ref.glob)
    ovf_ref = [k for k in range(top) if ref.glob_ovf[k]]
    assert res.overflow == ovf_ref
    for k in range(top):
        if not ref.glob_ovf[k]:
            assert res.counts[k] == ref.glob[k], (name, k, res.counts[k], ref.glob[k])
    assert all(c == 0 for c in res.counts[top:])
    assert res.omega == (min(ref.omega, kmax) if kmax else ref.omega)
    assert res.stats["alpha"] == ref.stats["alpha"]
    if not kmax:
        assert res.stats["leaves"] == ref.stats["leaves"], (res.stats, ref.stats)
        assert res.stats["nodes"] == ref.stats["nodes"], (res.stats, ref.stats)
        assert res.stats["work"] == ref.stats["work_sw"], (res.stats, ref.stats)
        # the roofline model's work terms: child formation and the leaves' additions
        assert res.stats["child_work"] == ref.stats["work_child"], (res.stats, ref.stats)
        assert res.stats["leaf_hp"] == ref.stats["leaf_hp"], (res.stats, ref.stats)
        hh, pp = np.indices(ref.hist.shape)
        assert res.stats["leaf_pp"] == int((ref.hist.astype(object) * (pp + 1)).sum())
    return res, ref


FAMILIES = [
    ("empty0", lambda: gg.empty(0)),
    ("empty5", lambda: gg.empty(5)),
    ("K1", lambda: gg.complete(1)),
    ("K2", lambda: gg.complete(2)),
    ("path9", lambda: gg.path(9)),
    ("star40", lambda: gg.star(40)),
    ("cycle11", lambda: gg.cycle(11)),
    ("K10", lambda: gg.complete(10)),
    ("K64", lambda: gg.complete(64)),
    ("K65", lambda: gg.complete(65)),
    ("K66", lambda: gg.complete(66)),
    ("K70", lambda: gg.complete(70)),
    ("K129", lambda: gg.complete(129)),
    ("multipartite", lambda: gg.complete_multipartite([1, 2, 3, 4, 5, 6, 7])),
    ("moon_moser8", lambda: gg.moon_moser(8)),
    ("cocktail12", lambda: gg.complete_multipartite([2] * 12)),
    ("wheel", lambda: gg.join(gg.cycle(9), gg.complete(1))),
]


@pytest.mark.parametrize("name,maker", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_families(ctx, name, maker):
    check_global(ctx, maker(), name)


@pytest.mark.parametrize("n", [132, 140])
def test_overflow_flags_match(ctx, n):
    res, ref = check_global(ctx, gg.complete(n), f"K{n}")
    assert res.status == P.PV_EOVERFLOW
    assert res.overflow and all(bool(ref.glob_ovf[k]) for k in res.overflow)


RANDOM = [(40, 0.3, 1), (90, 0.15, 2), (200, 0.05, 3), (120, 0.5, 4), (64, 0.8, 5)]


@pytest.mark.parametrize("n,p,seed", RANDOM)
def test_random_graphs(ctx, n, p, seed):
    check_global(ctx, gg.gnp(n, p, seed), f"gnp({n},{p},{seed})")


def test_er_planted_workload(ctx):
    # G(2000, 0.01) plus three planted 12-cliques: the small benchmark workload
    check_global(ctx, gg.er_planted(), "er2000+3xK12")


def test_heavy_roots_multiword(ctx):
    # planted cliques of 70..100 vertices give out-neighbourhoods > 64
    g = gg.plant_cliques(gg.gnp(600, 0.04, 7), [100, 80, 70], 8)
    res, ref = check_global(ctx, g, "gnp600+K100,K80,K70")
    assert ref.stats["alpha"] > 64


def test_heavy_dense_overlap(ctx):
    # dense random core with overlapping planted cliques: deep multi-word chains
    g = gg.plant_cliques(gg.gnp(160, 0.45, 11), [75, 40], 12)
    check_global(ctx, g, "gnp160(0.45)+K75,K40")


def test_chung_lu_medium(ctx):
    g = gg.chung_lu(20000, 20, 2.3, 2000, 5)
    check_global(ctx, g, "chung_lu 20k")


@pytest.mark.parametrize("kmax", [1, 2, 3, 5, 8])
def test_truncation(ctx, kmax):
    g = gg.plant_cliques(gg.gnp(300, 0.08, 21), [20, 15], 22)
    check_global(ctx, g, f"truncated kmax={kmax}", kmax=kmax)


@pytest.mark.parametrize("dfs_max", [1, 4, 16, 40, 64])
def test_split_threshold_does_not_change_the_tree(ctx, dfs_max):
    g = gg.plant_cliques(gg.gnp(400, 0.1, 31), [70, 30], 32)
    P.pv_set_dfs_max(ctx, dfs_max)
    try:
        check_global(ctx, g, f"dfs_max={dfs_max}")
    finally:
        P.pv_set_dfs_max(ctx, 64)


# --------------------------------------------------------------- per-vertex

LOCAL = [("gnp", lambda: gg.gnp(150, 0.2, 41), (1, 8)),
         ("planted", lambda: gg.plant_cliques(gg.gnp(300, 0.05, 42), [14, 9], 43), (3, 10)),
         ("heavy", lambda: gg.plant_cliques(gg.gnp(400, 0.04, 44), [90, 12], 45), (3, 10)),
         ("K40", lambda: gg.complete(40), (1, 16)),
         ("moon_moser", lambda: gg.moon_moser(7), (2, 7))]


@pytest.mark.parametrize("name,maker,krange", LOCAL, ids=[x[0] for x in LOCAL])
def test_per_vertex(ctx, name, maker, krange):
    g = maker()
    klo, khi = krange
    _say(f"[parity] per-vertex {name}: n={g.n} m={g.m} k={klo}..{khi}")
    with Loaded(ctx, g) as h:
        out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, klo, khi)
    ref = O.count(g, vertex=(klo, khi))
    assert ovf == 0
    assert np.array_equal(out, ref.vertex)


def test_combined_pass_with_device_output(ctx):
    import torch
    g = gg.plant_cliques(gg.chung_lu(5000, 16, 2.3, 800, 51), [40, 70], 52)
    klo, khi = 3, 10
    K = khi - klo + 1
    _say(f"[parity] combined pass n={g.n} m={g.m}")
    dev = torch.zeros((g.n, K, 2), dtype=torch.int64, device="cuda:0")
    with Loaded(ctx, g) as h:
        res, lovf = P.pv_count(h, reorient=True, local_kind=P.PV_VERTEX, k_lo=klo, k_hi=khi,
                               local_out=dev.data_ptr())
        sub = P.pv_graph_export_order(h)
    torch.cuda.synchronize()
    out = dev.cpu().numpy().view(np.uint64)
    ref = O.count(g, key=sub, vertex=(klo, khi))
    assert lovf == 0
    assert res.counts[: len(ref.glob)] == ref.glob
    assert res.stats["leaves"] == ref.stats["leaves"]
    assert np.array_equal(out, ref.vertex)


# ------------------------------------------------------------ root subsets

def test_root_subsets(ctx):
    g = gg.plant_cliques(gg.gnp(500, 0.06, 61), [80, 20], 62)
    rng = np.random.default_rng(63)
    with Loaded(ctx, g) as h:
        sub = P.pv_graph_export_order(h)
        roots = rng.choice(g.n, 120, replace=False).astype(np.int32)
        res = P.pv_count_roots(h, roots)
        empty = P.pv_count_roots(h, np.zeros(0, np.int32))
    ref = O.count(g, key=sub, roots=roots)
    assert res.counts[0] == 0
    assert res.counts[1: len(ref.glob)] == ref.glob[1:]
    assert res.stats["leaves"] == ref.stats["leaves"]
    assert all(c == 0 for c in empty.counts)


# -------------------------------------------------------------- validation

@pytest.mark.parametrize("bad", ["selfloop", "asym", "unsorted", "dup", "range"])
def test_invalid_csr_is_rejected(ctx, bad):
    rp = np.array([0, 2, 3, 4], dtype=np.int32)
    col = np.array([1, 2, 0, 0], dtype=np.int32)  # 0-1, 0-2 ok
    if bad == "selfloop":
        col = np.array([0, 2, 0, 0], dtype=np.int32)
    elif bad == "asym":
        rp = np.array([0, 2, 3, 3], dtype=np.int32)
        col = np.array([1, 2, 0], dtype=np.int32)
    elif bad == "unsorted":
        col = np.array([2, 1, 0, 0], dtype=np.int32)
    elif bad == "dup":
        rp = np.array([0, 2, 4, 5], dtype=np.int32)
        col = np.array([1, 1, 0, 0, 0], dtype=np.int32)
    elif bad == "range":
        col = np.array([1, 7, 0, 0], dtype=np.int32)
    with pytest.raises(P.PivoterError) as ei:
        h = P.pv_graph_load_csr(ctx, 3, rp, col)
        P.pv_graph_free(h)
    assert ei.value.status == P.PV_ENOTSIMPLE


def test_valid_tiny_csr_is_accepted(ctx):
    rp = np.array([0, 2, 3, 4], dtype=np.int32)
    col = np.array([1, 2, 0, 0], dtype=np.int32)
    h = P.pv_graph_load_csr(ctx, 3, rp, col)
    res = P.pv_count_global(h)
    P.pv_graph_free(h)
    assert res.counts[:4] == [1, 3, 2, 0]


# --------------------------------------------------- peel at larger sizes

@pytest.mark.parametrize("n,deg,seed", [(12000, 12, 71), (20000, 10, 73), (200000, 16, 72)])
def test_peel_order_large(ctx, n, deg, seed):
    # one-block phase only (12000), a few grid sub-rounds first (20000), and
    # a long grid-wide phase (200000)
    g = gg.chung_lu(n, deg, 2.3, n // 20, seed)
    _say(f"[parity] peel n={g.n} m={g.m}")
    with Loaded(ctx, g) as h:
        alpha = P.pv_graph_orient(h)
        sub = P.pv_graph_export_order(h)
    pe = O.peel(g)
    assert alpha == pe.alpha
    assert np.array_equal(sub, pe.sub)


@pytest.mark.parametrize("n", [16384, 16385, 65536])
def test_peel_order_with_a_hub(ctx, n):
    # a vertex adjacent to all others: remaining degrees up to n - 1 in the
    # one-block phase (its largest size), just past it, and far past it
    g0 = gg.chung_lu(n, 6, 2.3, 500, 74)
    hub = np.arange(1, n, dtype=np.int64)
    ia, ja = g0.edges()
    g = gg.from_edges(n, np.concatenate([ia, np.zeros_like(hub)]), np.concatenate([ja, hub]))
    _say(f"[parity] peel with hub n={g.n} m={g.m}")
    with Loaded(ctx, g) as h:
        alpha = P.pv_graph_orient(h)
        sub = P.pv_graph_export_order(h)
    pe = O.peel(g)
    assert alpha == pe.alpha
    assert np.array_equal(sub, pe.sub)


def _paths(lengths):
    g = gg.path(int(lengths[0]))
    for L in lengths[1:]:
        g = gg.disjoint_union(g, gg.path(int(L)))
    return g


@pytest.mark.parametrize("name,g", [("path 40000", gg.path(40_000)),
                                    ("paths 2..300 and 60000", _paths(np.append(np.arange(2, 301), 60_000)))])
def test_peel_order_small_frontiers(ctx, name, g):
    # long runs of sub-rounds with a handful of vertices each while the
    # graph is still large: the runs block 0 takes alone between two grid
    # barriers (frontiers of a path shrink to two vertices; a union of paths
    # goes from large frontiers to small ones as its shorter paths run out)
    _say(f"[parity] peel {name} n={g.n}")
    with Loaded(ctx, g) as h:
        alpha = P.pv_graph_orient(h)
        sub = P.pv_graph_export_order(h)
    pe = O.peel(g)
    assert alpha == pe.alpha
    assert np.array_equal(sub, pe.sub)


@pytest.mark.parametrize("name,g", [("cycle 16384", gg.cycle(16384)), ("cycle 40000", gg.cycle(40000)),
                                    ("empty 30000", gg.empty(30000))])
def test_peel_order_one_big_frontier(ctx, name, g):
    # every vertex leaves in the first sub-round: the largest frontier the
    # one-block phase holds, and whole-graph frontiers in the grid phase
    _say(f"[parity] peel {name}")
    with Loaded(ctx, g) as h:
        alpha = P.pv_graph_orient(h)
        sub = P.pv_graph_export_order(h)
    pe = O.peel(g)
    assert alpha == pe.alpha
    assert np.array_equal(sub, pe.sub)


# ------------------------------------------------------------- lane tier

LANE_GRAPHS = [
    ("gnp 300 0.1", lambda: gg.gnp(300, 0.1, 95)),
    ("planted 400", lambda: gg.plant_cliques(gg.gnp(400, 0.05, 96), [14, 9, 8, 8], 97)),
    ("chung-lu 3000", lambda: gg.chung_lu(3000, 16, 2.2, 300, 98)),
    ("multipartite", lambda: gg.complete_multipartite([2] * 12)),
]


def _local_run(ctx, g, lane_max, budget=2048):
    P.pv_set_lane_max(ctx, lane_max)
    P.pv_set_dfs_budget(ctx, budget)
    try:
        with Loaded(ctx, g) as h:
            out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, 3, 10)
            tr = P.pv_count_global(h, k_max=5)
    finally:
        P.pv_set_lane_max(ctx, 8)
        P.pv_set_dfs_budget(ctx, 0)
    return out, ovf, st, tr


@pytest.mark.parametrize("lane_max", [3, 8])
@pytest.mark.parametrize("name,make", LANE_GRAPHS)
def test_lane_tier_keeps_tree_and_counts(ctx, name, make, lane_max):
    # subtrees of at most lane_max vertices walked one per lane: the same
    # tree (node, leaf and work counts) and the same global and per-vertex
    # counts, also on truncated trees (local counts for k <= 10 walk the tree
    # truncated at 10 holds; there the oracle walks the rest of a truncated
    # pivot chain node by node, so node counts are compared with the
    # wave-only walk) and with depth-first splits between the batches
    g = make()
    _say(f"[parity] lane tier {name} lane_max={lane_max}")
    P.pv_set_lane_max(ctx, lane_max)
    try:
        check_global(ctx, g, f"{name} lane_max={lane_max}")
        check_global(ctx, g, f"{name} lane_max={lane_max}", kmax=5, check_order=False)
    finally:
        P.pv_set_lane_max(ctx, 8)
    ref = O.count(g, vertex=(3, 10))
    w_out, w_ovf, w_st, w_tr = _local_run(ctx, g, 0)
    assert w_ovf == 0 and np.array_equal(w_out, ref.vertex)
    for budget in (2048, 16):
        out, ovf, st, tr = _local_run(ctx, g, lane_max, budget)
        assert ovf == 0 and np.array_equal(out, ref.vertex), budget
        for key in ("nodes", "leaves", "work"):
            assert st[key] == w_st[key], (key, budget, st[key], w_st[key])
            assert tr.stats[key] == w_tr.stats[key], (key, budget)
        assert tr.counts == w_tr.counts


# ------------------------------------------------ local counts for all k

ALLK_GRAPHS = [
    ("K30", lambda: gg.complete(30)),
    ("planted 300", lambda: gg.plant_cliques(gg.gnp(300, 0.05, 171), [26, 19], 172)),
    ("multipartite 3x11", lambda: gg.complete_multipartite([3] * 11)),
]


@pytest.mark.parametrize("name,make", ALLK_GRAPHS)
def test_local_counts_for_all_k(ctx, name, make):
    # k ranges wider than one walk's slots go window by window (16 values
    # per vertex, 8 per edge), including windows that start above k = 16
    g = make()
    with Loaded(ctx, g) as h:
        res = P.pv_count_global(h)
        w = res.omega + 2
        _say(f"[parity] all-k local counts {name}: omega={res.omega}, k=1..{w}")
        vout, vovf, _ = P.pv_count_local(h, P.PV_VERTEX, 1, w)
        eout, eovf, _ = P.pv_count_local(h, P.PV_EDGE, 2, w)
        hi_v = P.pv_count_local(h, P.PV_VERTEX, 17, w) if w >= 17 else None
    ref = O.count(g, vertex=(1, w), edge=(2, w))
    assert vovf == 0 and eovf == 0
    assert np.array_equal(vout, ref.vertex)
    assert np.array_equal(eout, ref.edge)
    if hi_v is not None:
        assert hi_v[1] == 0 and np.array_equal(hi_v[0], ref.vertex[:, 16:])


# ---------------------------------------------- forced depth-first splits

SPLITS = [(32, 16), (8, 16), (64, 24), (64, 1 << 20)]


@pytest.mark.parametrize("dfs_max,budget", SPLITS)
def test_dfs_budget_splits_keep_the_tree(ctx, dfs_max, budget):
    g = gg.plant_cliques(gg.gnp(400, 0.12, 91), [75, 30, 20], 92)
    P.pv_set_dfs_max(ctx, dfs_max)
    P.pv_set_dfs_budget(ctx, budget)
    try:
        res, ref = check_global(ctx, g, f"dfs_max={dfs_max} budget={budget}")
        with Loaded(ctx, g) as h:
            out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, 3, 10)
        vref = O.count(g, vertex=(3, 10))
        assert ovf == 0 and np.array_equal(out, vref.vertex)
    finally:
        P.pv_set_dfs_max(ctx, 64)
        P.pv_set_dfs_budget(ctx, 0)


# ----------------------------------------------------------------- per-edge

EDGE = [("gnp", lambda: gg.gnp(150, 0.2, 141), (1, 8)),
        ("planted", lambda: gg.plant_cliques(gg.gnp(300, 0.05, 142), [14, 9], 143), (3, 10)),
        ("heavy", lambda: gg.plant_cliques(gg.gnp(400, 0.04, 144), [90, 12], 145), (3, 8)),
        ("heavy_dense", lambda: gg.plant_cliques(gg.gnp(160, 0.45, 146), [75, 40], 147), (2, 6)),
        ("K40", lambda: gg.complete(40), (2, 9)),
        ("multipartite", lambda: gg.complete_multipartite([1, 2, 3, 4, 5, 6, 7]), (1, 7)),
        ("moon_moser", lambda: gg.moon_moser(7), (2, 7)),
        ("star", lambda: gg.star(30), (1, 4)),
        ("empty", lambda: gg.empty(6), (2, 4))]


@pytest.mark.parametrize("name,maker,krange", EDGE, ids=[x[0] for x in EDGE])
def test_per_edge(ctx, name, maker, krange):
    g = maker()
    klo, khi = krange
    _say(f"[parity] per-edge {name}: n={g.n} m={g.m} k={klo}..{khi}")
    with Loaded(ctx, g) as h:
        out, ovf, st = P.pv_count_local(h, P.PV_EDGE, klo, khi)
        eu, ev = P.pv_graph_edge_list(h)
    ref = O.count(g, edge=(klo, khi))
    a, b = g.edges()
    assert np.array_equal(eu, a) and np.array_equal(ev, b)
    assert ovf == 0
    assert np.array_equal(out, ref.edge)


@pytest.mark.parametrize("dfs_max,budget", [(8, 16), (64, 24), (16, 1 << 20)])
def test_per_edge_splits(ctx, dfs_max, budget):
    g = gg.plant_cliques(gg.gnp(400, 0.12, 191), [75, 30, 20], 192)
    P.pv_set_dfs_max(ctx, dfs_max)
    P.pv_set_dfs_budget(ctx, budget)
    try:
        _say(f"[parity] per-edge splits dfs_max={dfs_max} budget={budget}")
        with Loaded(ctx, g) as h:
            out, ovf, st = P.pv_count_local(h, P.PV_EDGE, 3, 8)
        ref = O.count(g, edge=(3, 8))
        assert ovf == 0 and np.array_equal(out, ref.edge)
    finally:
        P.pv_set_dfs_max(ctx, 64)
        P.pv_set_dfs_budget(ctx, 0)


def test_per_edge_combined_device_output(ctx):
    import torch
    g = gg.plant_cliques(gg.chung_lu(5000, 16, 2.3, 800, 151), [40, 70], 152)
    klo, khi = 3, 8
    K = khi - klo + 1
    _say(f"[parity] per-edge combined pass n={g.n} m={g.m}")
    dev = torch.zeros((g.m, K, 2), dtype=torch.int64, device="cuda:0")
    with Loaded(ctx, g) as h:
        res, lovf = P.pv_count(h, reorient=True, local_kind=P.PV_EDGE, k_lo=klo, k_hi=khi,
                               local_out=dev.data_ptr())
        sub = P.pv_graph_export_order(h)
    torch.cuda.synchronize()
    out = dev.cpu().numpy().view(np.uint64)
    ref = O.count(g, key=sub, edge=(klo, khi))
    assert lovf == 0
    assert res.counts[: len(ref.glob)] == ref.glob
    assert np.array_equal(out, ref.edge)


def test_per_edge_wide_range(ctx):
    # one walk keeps 8 per-edge k-slots: pv_count refuses a wider range,
    # pv_count_local covers it window by window
    import torch
    g = gg.gnp(50, 0.2, 161)
    with Loaded(ctx, g) as h:
        dev = torch.zeros((g.m, 9, 2), dtype=torch.int64, device="cuda:0")
        with pytest.raises(P.PivoterError) as ei:
            P.pv_count(h, local_kind=P.PV_EDGE, k_lo=2, k_hi=10, local_out=dev.data_ptr())
        out, ovf, _ = P.pv_count_local(h, P.PV_EDGE, 2, 10)
    assert ei.value.status == P.PV_EINVAL
    assert ovf == 0 and np.array_equal(out, O.count(g, edge=(2, 10)).edge)


# Local counts added in packed 32-bit halves (counts below 2^62): per edge the
# pair charges, per vertex the members' sums.  A starting value just under
# 2^32 makes both halves of a word wrap after a few additions, so the carry
# bookkeeping is exercised on small graphs; with packing off the additions
# go straight to the output.  All must give the oracle's counts.
PACKED = [("heavy", lambda: gg.plant_cliques(gg.gnp(400, 0.04, 144), [90, 12], 145), (3, 8)),
          ("gnp_odd_K", lambda: gg.gnp(150, 0.2, 141), (1, 5)),
          ("K40", lambda: gg.complete(40), (2, 9)),
          ("K40_16k", lambda: gg.complete(40), (1, 16))]


@pytest.mark.parametrize("env", [{"PV_PACK_BIAS": "0xfffffffa"}, {"PV_PACK_BIAS": "0xffffffff"},
                                 {"PV_PACK": "0"}], ids=["bias_fffffffa", "bias_ffffffff", "unpacked"])
@pytest.mark.parametrize("kind", [P.PV_EDGE, P.PV_VERTEX], ids=["edge", "vertex"])
@pytest.mark.parametrize("name,maker,krange", PACKED, ids=[x[0] for x in PACKED])
def test_local_counts_packed_halves(monkeypatch, env, kind, name, maker, krange):
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    g = maker()
    klo, khi = krange
    what = "edge" if kind == P.PV_EDGE else "vertex"
    _say(f"[parity] per-{what} {name} {env}: n={g.n} m={g.m} k={klo}..{khi}")
    c = P.pv_init(0)
    try:
        with Loaded(c, g) as h:
            out, ovf, st = P.pv_count_local(h, kind, klo, khi)
    finally:
        P.pv_fini(c)
    ref = O.count(g, **{what: (klo, khi)})
    assert ovf == 0
    assert np.array_equal(out, ref.edge if kind == P.PV_EDGE else ref.vertex)


# ------------------------------------------------------------------ batches

def _check_batch(ctx, graphs, kmax=0, tag=""):
    _say(f"[parity] batch {tag}: {len(graphs)} graphs kmax={kmax}")
    hs = [P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col) for g in graphs]
    try:
        res, st = P.pv_count_global_batch(ctx, hs, k_max=kmax)
        single = [P.pv_count_global(h, kmax) for h in hs]
    finally:
        for h in hs:
            P.pv_graph_free(h)
    leaves = 0
    for i, g in enumerate(graphs):
        ref = O.count(g, kmax=kmax)
        top = len(ref.glob)
        ovf_ref = [k for k in range(top) if ref.glob_ovf[k]]
        assert res[i].overflow == ovf_ref, (tag, i)
        for k in range(top):
            if not ref.glob_ovf[k]:
                assert res[i].counts[k] == ref.glob[k], (tag, i, k)
        assert all(c == 0 for c in res[i].counts[top:])
        assert res[i].omega == (min(ref.omega, kmax) if kmax else ref.omega)
        # the batch walks the same trees as one call per graph
        assert res[i].counts[:top] == single[i].counts[:top] and res[i].omega == single[i].omega
        leaves += ref.stats["leaves"]
    if not kmax:
        assert st["leaves"] == leaves
    return res


MIXED = [gg.empty(0), gg.empty(5), gg.complete(1), gg.complete(10), gg.gnp(40, 0.3, 301),
         gg.plant_cliques(gg.gnp(600, 0.04, 302), [100, 80, 70], 303), gg.moon_moser(6),
         gg.chung_lu(2000, 12, 2.5, 200, 304), gg.star(25), gg.cycle(9), gg.complete(66)]


def test_batch_mixed(ctx):
    _check_batch(ctx, MIXED, tag="mixed")


@pytest.mark.parametrize("kmax", [3, 6])
def test_batch_truncated(ctx, kmax):
    _check_batch(ctx, MIXED, kmax=kmax, tag="mixed truncated")


def test_batch_overflow_flags_are_per_graph(ctx):
    res = _check_batch(ctx, [gg.complete(20), gg.complete(133), gg.gnp(50, 0.2, 305)], tag="ovf")
    assert res[0].overflow == [] and res[2].overflow == []
    assert res[1].overflow


def test_batch_workload_whole(ctx):
    # the whole 4096-graph batch workload in one union pass, as the
    # benchmark runs it: every member against one call per graph, and every
    # 16th member (256 graphs spread over the size range) against the oracle
    specs = gg.batch_graph_specs()
    graphs = [gg.chung_lu(n, d, 2.5, n - 1, s) for (n, d, s) in specs]
    _say(f"[parity] batch workload: {len(graphs)} graphs, m={sum(g.m for g in graphs)}")
    hs = [P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col) for g in graphs]
    try:
        res, st = P.pv_count_global_batch(ctx, hs)
        single = [P.pv_count_global(h) for h in hs]
    finally:
        for h in hs:
            P.pv_graph_free(h)
    for i, (r, s1) in enumerate(zip(res, single)):
        # (the two calls return count buffers of different lengths, zero past omega)
        top = min(len(r.counts), len(s1.counts))
        assert r.counts[:top] == s1.counts[:top] and not any(r.counts[top:]) and not any(s1.counts[top:]), i
        assert r.omega == s1.omega and r.omega < top and r.overflow == s1.overflow == [], i
    assert st["leaves"] == sum(s1.stats["leaves"] for s1 in single)
    for i in range(0, len(graphs), 16):
        ref = O.count(graphs[i])
        assert res[i].counts[: len(ref.glob)] == ref.glob, i
        assert all(c == 0 for c in res[i].counts[len(ref.glob):]) and res[i].omega == ref.omega, i


def test_batch_reuses_union_buffers(ctx):
    # a second, smaller batch on the same context after a larger one
    _check_batch(ctx, MIXED, tag="first")
    _check_batch(ctx, MIXED[:4], tag="second")


@pytest.mark.parametrize("khi", [8, 15])
def test_per_vertex_wide_and_narrow_sums(ctx, khi):
    # K_100 with k up to 15: C(99, 14) * (budget + 256) exceeds 2^64, so the
    # per-visit sums take the 128-bit path; up to 8 they take the 64-bit one
    g = gg.plant_cliques(gg.gnp(300, 0.05, 171), [100], 172)
    _say(f"[parity] per-vertex k=1..{khi} on gnp300+K100")
    with Loaded(ctx, g) as h:
        out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, 1, khi)
    ref = O.count(g, vertex=(1, khi))
    assert ovf == 0
    assert np.array_equal(out, ref.vertex)


@pytest.mark.parametrize("kmax", [2, 4, 7, 11])
def test_truncation_heavy_roots(ctx, kmax):
    # multi-word roots (a planted K_90) under truncation: the walk stops at
    # k_max hold vertices in every tier
    g = gg.plant_cliques(gg.gnp(500, 0.06, 181), [90, 30], 182)
    check_global(ctx, g, f"heavy truncated kmax={kmax}", kmax=kmax)
    with Loaded(ctx, g) as h:
        out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, 2, kmax)
        eout, eovf, _ = P.pv_count_local(h, P.PV_EDGE, 2, min(kmax, 9))
    ref = O.count(g, vertex=(2, kmax), edge=(2, min(kmax, 9)))
    assert ovf == 0 and np.array_equal(out, ref.vertex)
    assert eovf == 0 and np.array_equal(eout, ref.edge)


# ------------------------------------- heavy roots: prefix sums and chunks

def _ctx_env(**env):
    """A fresh context created while the given environment variables are set."""
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return P.pv_init(0)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


HEAVY = [("heavy", lambda: gg.plant_cliques(gg.gnp(400, 0.04, 44), [90, 12], 45), (3, 10)),
         ("heavy_dense", lambda: gg.plant_cliques(gg.gnp(160, 0.45, 146), [75, 40], 147), (2, 9)),
         ("K129", lambda: gg.complete(129), (1, 16))]
_HEAVY_REF = {}


def _heavy_case(name):
    if name not in _HEAVY_REF:
        maker, (klo, khi) = {x[0]: (x[1], x[2]) for x in HEAVY}[name]
        g = maker()
        ref = O.count(g, vertex=(klo, khi), edge=(2, min(khi, 6)))
        _HEAVY_REF[name] = (g, klo, khi, ref)
    return _HEAVY_REF[name]


@pytest.mark.parametrize("rows", [1, 7, 0])
@pytest.mark.parametrize("name", [x[0] for x in HEAVY])
def test_per_vertex_prefix_passes(name, rows):
    # what the universes of a heavy root owe the vertices above them is
    # summed per heavy root on chip, `rows` vertices of N+(root) per pass
    # (0: as many as fit); any pass size gives the same counts
    g, klo, khi, ref = _heavy_case(name)
    _say(f"[parity] per-vertex prefix passes {name}: n={g.n} m={g.m} k={klo}..{khi} rows={rows}")
    c = _ctx_env(PV_PREFIX_ROWS=rows)
    try:
        with Loaded(c, g) as h:
            out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, klo, khi)
    finally:
        P.pv_fini(c)
    assert ovf == 0
    assert np.array_equal(out, ref.vertex)


@pytest.mark.parametrize("name", [x[0] for x in HEAVY])
def test_heavy_roots_in_chunks(name):
    # a 1-byte budget for gathered neighbourhoods takes the heavy roots one
    # per chunk: global, per-vertex and per-edge results are unchanged
    g, klo, khi, ref = _heavy_case(name)
    _say(f"[parity] heavy roots one per chunk {name}: n={g.n} m={g.m}")
    c = _ctx_env(PV_HU_BUDGET=1)
    try:
        with Loaded(c, g) as h:
            res = P.pv_count_global(h, 0)
            out, ovf, st = P.pv_count_local(h, P.PV_VERTEX, klo, khi)
            eout, eovf, est = P.pv_count_local(h, P.PV_EDGE, 2, min(khi, 6))
    finally:
        P.pv_fini(c)
    top = len(ref.glob)
    assert [res.counts[k] for k in range(top)] == [int(x) for x in ref.glob]
    assert res.stats["nodes"] == ref.stats["nodes"] and res.stats["leaves"] == ref.stats["leaves"]
    assert ovf == 0 and eovf == 0
    assert np.array_equal(out, ref.vertex)
    assert np.array_equal(eout, ref.edge)


# ----------------------------------------------- counts wider than 128 bits

def _esym(parts):
    e = [1]
    for a in parts:
        e = [x + (a * e[i - 1] if i else 0) for i, x in enumerate(e + [0])]
    return e


WIDE = [("K200", lambda: gg.complete(200), 4),
        ("K300", lambda: gg.complete(300), 5),
        ("multipartite153", lambda: gg.complete_multipartite([1] * 150 + [2, 3, 3]), 3),
        ("planted160", lambda: gg.plant_cliques(gg.gnp(600, 0.02, 61), [160, 130], 62), 3)]


@pytest.mark.parametrize("name,maker,limbs", WIDE, ids=[w[0] for w in WIDE])
def test_wide_counts(ctx, name, maker, limbs):
    from math import comb
    g = maker()
    _say(f"[parity] wide counts {name}: n={g.n} m={g.m} limbs={limbs}")
    if name.startswith("K"):
        want, omega = [comb(g.n, k) for k in range(g.n + 1)], g.n
    elif name.startswith("multipartite"):
        want = _esym([1] * 150 + [2, 3, 3])
        omega = len(want) - 1
    else:
        want, omega = O.counts_exact(g)
    with Loaded(ctx, g) as h:
        res = P.pv_count_global_wide(h, 0, cap=omega + 2, limbs=limbs)
    assert res.status == P.PV_OK and res.overflow == []
    assert res.omega == omega
    assert res.counts[: omega + 1] == want and res.counts[omega + 1] == 0
    assert max(want) >= 2 ** 128 or name.startswith("planted")


@pytest.mark.parametrize("limbs", [1, 2])
def test_wide_counts_narrow_limbs_flag_overflow(ctx, limbs):
    # K_200 in 64 or 128 bits: exactly the C(200, k) that do not fit are
    # flagged, and their limbs hold the count modulo 2^(64 limbs)
    from math import comb
    g = gg.complete(200)
    with Loaded(ctx, g) as h:
        res = P.pv_count_global_wide(h, 0, cap=202, limbs=limbs)
    mod = 2 ** (64 * limbs)
    assert res.status == P.PV_EOVERFLOW
    assert res.overflow == [k for k in range(202) if k <= 200 and comb(200, k) >= mod]
    assert res.counts[:201] == [comb(200, k) % mod for k in range(201)]


def test_wide_counts_agree_with_u128_truncation_and_tiny_graphs(ctx):
    from math import comb
    g = gg.plant_cliques(gg.gnp(400, 0.05, 71), [45, 30], 72)
    with Loaded(ctx, g) as h:
        a = P.pv_count_global(h)
        b = P.pv_count_global_wide(h, 0, limbs=2)
        t = P.pv_count_global_wide(h, 12, limbs=2)
        ta = P.pv_count_global(h, 12)
    assert b.counts == a.counts and b.omega == a.omega and b.overflow == a.overflow == []
    assert b.stats["leaves"] == a.stats["leaves"] and b.stats["nodes"] == a.stats["nodes"]
    assert t.counts == ta.counts and t.omega == ta.omega
    with Loaded(ctx, gg.complete(200)) as h:
        r = P.pv_count_global_wide(h, 20, cap=202, limbs=4)
    assert r.counts[:21] == [comb(200, k) for k in range(21)] and all(c == 0 for c in r.counts[21:])
    for gt, want in [(gg.empty(0), [1]), (gg.empty(5), [1, 5]), (gg.complete(1), [1, 1])]:
        with Loaded(ctx, gt) as h:
            r = P.pv_count_global_wide(h, 0, cap=4, limbs=1)
        assert r.counts == want + [0] * (4 - len(want)), (gt.n, r.counts)


# ---------------------------------------- frequency distributions f_k(b)

def test_local_frequency_per_vertex_and_per_edge(ctx):
    import torch
    g = gg.plant_cliques(gg.gnp(400, 0.05, 81), [30, 18], 82)
    klo, khi = 3, 10
    K = khi - klo + 1
    ref = O.count(g, vertex=(klo, khi), edge=(3, 8))
    loc = torch.zeros((g.n, K, 2), dtype=torch.int64, device="cuda:0")
    with Loaded(ctx, g) as h:
        P.pv_count(h, reorient=True, local_kind=P.PV_VERTEX, k_lo=klo, k_hi=khi, local_out=loc.data_ptr())
        torch.cuda.synchronize()
        eout, eovf, est = P.pv_count_local(h, P.PV_EDGE, 3, 8)
    for c in range(K):
        vals, freq = P.pv_local_frequency(ctx, loc.data_ptr(), g.n, K, c)
        assert list(zip(vals, (int(f) for f in freq))) == O.frequency(ref.vertex[:, c]), c
    ed = torch.from_numpy(eout.view(np.int64).copy()).to("cuda:0")
    for c in range(6):
        vals, freq = P.pv_local_frequency(ctx, ed.data_ptr(), g.m, 6, c)
        assert list(zip(vals, (int(f) for f in freq))) == O.frequency(ref.edge[:, c]), c
    # no rows, one row, and a buffer too small for the distinct values
    vals, freq = P.pv_local_frequency(ctx, loc.data_ptr(), 0, K, 0)
    assert vals == [] and len(freq) == 0
    vals, freq = P.pv_local_frequency(ctx, loc.data_ptr(), 1, K, 0)
    assert len(vals) == 1 and int(freq[0]) == 1
    import ctypes as C
    one_v = (P.pv_u128 * 1)()
    one_f = (C.c_uint64 * 1)()
    nd = C.c_int64()
    st = P.load_library().pv_local_frequency(ctx, loc.data_ptr(), g.n, K, 0, one_v, one_f, 1, C.byref(nd))
    assert st == P.PV_EBUFSIZE and nd.value == len(O.frequency(ref.vertex[:, 0])) > 1
