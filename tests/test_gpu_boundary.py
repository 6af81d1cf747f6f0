"""The C-ABI boundary on the GPU: input repair, the device-memory budget, the
in-use refusal of pv_graph_free, per-graph batch statuses, the tuning cache,
and local counts of root subsets.  Every count is checked against the oracle.
"""
import json
import sys
import threading
import time

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


def _global(ctx, g, flags=0, row_ptr=None, col=None):
    rp = g.row_ptr if row_ptr is None else row_ptr
    cl = g.col if col is None else col
    h = P.pv_graph_load_csr(ctx, g.n, rp, cl, flags)
    try:
        return P.pv_count_global(h), P.pv_graph_size(h)
    finally:
        P.pv_graph_free(h)


# ------------------------------------------------------------ input repair

def _messy(g, seed):
    """each undirected edge once in a random direction, plus repeats and
    self loops, rows unsorted: a directed multigraph CSR"""
    rng = np.random.default_rng(seed)
    a, b = g.edges()
    flip = rng.random(len(a)) < 0.5
    src = np.where(flip, b, a)
    dst = np.where(flip, a, b)
    rep = rng.choice(len(a), len(a) // 5, replace=False)
    loops = rng.choice(g.n, 10, replace=False)
    src = np.concatenate([src, src[rep], loops])
    dst = np.concatenate([dst, dst[rep], loops])
    perm = rng.permutation(len(src))
    src, dst = src[perm], dst[perm]
    order = np.argsort(src, kind="stable")
    rp = np.zeros(g.n + 1, dtype=np.int32)
    np.add.at(rp, src + 1, 1)
    return np.cumsum(rp).astype(np.int32), dst[order].astype(np.int32)


def test_symmetrize_repairs_a_directed_multigraph(ctx):
    g = gg.plant_cliques(gg.gnp(300, 0.04, 31), [14, 9], 32)
    rp, col = _messy(g, 33)
    h = None
    with pytest.raises(P.PivoterError) as ei:
        h = P.pv_graph_load_csr(ctx, g.n, rp, col)
    assert ei.value.status == P.PV_ENOTSIMPLE and h is None
    res, (n, m) = _global(ctx, g, P.PV_SYMMETRIZE, rp, col)
    ref = O.count(g)
    assert (n, m) == (g.n, g.m)
    assert res.counts[: len(ref.glob)] == ref.glob and res.omega == ref.omega


def test_dedup_repairs_repeats_loops_and_row_order(ctx):
    g = gg.gnp(200, 0.08, 34)
    rng = np.random.default_rng(35)
    rows = []
    for v in range(g.n):
        r = list(g.col[g.row_ptr[v]:g.row_ptr[v + 1]])
        r += r[: len(r) // 3] + [v]  # repeats and a self loop
        rng.shuffle(r)
        rows.append(r)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    col = np.concatenate(rows).astype(np.int32)
    res, (n, m) = _global(ctx, g, P.PV_DEDUP, rp, col)
    ref = O.count(g)
    assert m == g.m and res.counts[: len(ref.glob)] == ref.glob


def test_repair_of_a_device_csr(ctx):
    import torch
    g = gg.plant_cliques(gg.gnp(150, 0.05, 36), [11], 37)
    rp, col = _messy(g, 38)
    drp = torch.from_numpy(rp).to("cuda:0")
    dcol = torch.from_numpy(col).to("cuda:0")
    h = P.pv_graph_load_csr_device(ctx, g.n, len(col), drp.data_ptr(), dcol.data_ptr(), P.PV_SYMMETRIZE)
    try:
        res = P.pv_count_global(h)
        assert P.pv_graph_size(h) == (g.n, g.m)
    finally:
        P.pv_graph_free(h)
    assert res.counts[: len(O.count(g).glob)] == O.count(g).glob


def test_repair_refuses_ids_out_of_range(ctx):
    rp = np.array([0, 1, 2], dtype=np.int32)
    col = np.array([1, 5], dtype=np.int32)
    with pytest.raises(P.PivoterError) as ei:
        P.pv_graph_load_csr(ctx, 2, rp, col, P.PV_SYMMETRIZE)
    assert ei.value.status == P.PV_ENOTSIMPLE


# ------------------------------------------------------- memory budget

def test_budget_refuses_then_context_stays_usable():
    big = gg.chung_lu(200_000, 12, 2.3, 3000, 39)
    csr = 4 * (big.n + 1) + 8 * big.m
    budget = csr + (6 << 20)  # the graph fits, its walk's workspace does not
    c = P.pv_init(0, hbm_budget=budget)
    try:
        h = P.pv_graph_load_csr(c, big.n, big.row_ptr, big.col)
        assert P.pv_memory(c) <= budget
        with pytest.raises(P.PivoterError) as ei:
            P.pv_count_global(h)
        assert ei.value.status == P.PV_ENOMEM
        assert P.pv_memory(c) <= budget
        P.pv_graph_free(h)
        too_big = gg.chung_lu(2_000_000, 12, 2.3, 3000, 40)
        with pytest.raises(P.PivoterError) as ei:
            P.pv_graph_load_csr(c, too_big.n, too_big.row_ptr, too_big.col)
        assert ei.value.status == P.PV_ENOMEM
        small = gg.plant_cliques(gg.gnp(400, 0.03, 41), [13], 42)
        res, _ = _global(c, small)
        assert res.counts[: len(O.count(small).glob)] == O.count(small).glob
        assert P.pv_memory(c) <= budget
    finally:
        P.pv_fini(c)


def test_per_edge_packed_tables_give_way_to_the_budget(monkeypatch):
    # the packed per-edge tables (2 x m x 4 words here) are an option: a
    # budget that holds the unpacked walk but not them still gives the
    # oracle's counts, with the charges sent straight to the output
    g = gg.plant_cliques(gg.chung_lu(20000, 14, 2.3, 800, 611), [30], 612)
    ref = O.count(g, edge=(3, 8))
    tables = 2 * g.m * 4 * 8
    monkeypatch.setenv("PV_PACK", "0")
    c0 = P.pv_init(0)
    try:
        h = P.pv_graph_load_csr(c0, g.n, g.row_ptr, g.col)
        out0, ovf0, _ = P.pv_count_local(h, P.PV_EDGE, 3, 8)
        need = P.pv_memory(c0)
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c0)
    monkeypatch.delenv("PV_PACK")
    budget = need + (2 << 20)
    assert budget < need + tables
    _say(f"[boundary] per-edge under a budget: m={g.m} unpacked walk holds {need} bytes, budget {budget}")
    c = P.pv_init(0, hbm_budget=budget)
    try:
        h = P.pv_graph_load_csr(c, g.n, g.row_ptr, g.col)
        out, ovf, _ = P.pv_count_local(h, P.PV_EDGE, 3, 8)
        assert P.pv_memory(c) <= budget
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c)
    assert ovf0 == 0 and np.array_equal(out0, ref.edge)
    assert ovf == 0 and np.array_equal(out, ref.edge)


# -------------------------------------------- a graph in use is not freed

def test_free_refuses_a_graph_in_use(ctx):
    import torch
    g = gg.chung_lu_social(n=1_000_000, avg_deg=20.0, gamma=2.3, max_deg=20_000.0, seed=1)
    c2 = P.pv_init(0)
    h = P.pv_graph_load_csr(c2, g.n, g.row_ptr, g.col)
    out = {}

    def run():
        out["local"] = P.pv_count_local(h, P.PV_EDGE, 3, 8)  # about a second

    t = threading.Thread(target=run)
    t.start()
    time.sleep(0.3)
    saw = []
    while t.is_alive():
        st = P.pv_graph_free(h)
        assert st == P.PV_EAGAIN, st  # never released while counting
        saw.append(st)
        time.sleep(0.05)
    t.join()
    assert saw, "the count ended before the first free call"
    res = P.pv_count_global(h, k_max=3)  # the graph is intact
    assert P.pv_graph_free(h) == P.PV_OK
    P.pv_fini(c2)
    _say(f"[boundary] {len(saw)} refused frees during the count")
    # per-edge c_3 sums to 3 C_3 (each triangle has three edges)
    e3 = out["local"][0][:, 0, :]
    total = int(e3[:, 0].astype(object).sum()) + (int(e3[:, 1].astype(object).sum()) << 64)
    assert total == 3 * res.counts[3]


# ------------------------------------------------ per-graph batch status

def test_batch_reports_each_graphs_status(ctx):
    graphs = [gg.complete(5), gg.complete(12), gg.empty(3), gg.gnp(40, 0.2, 43)]
    hs = [P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col) for g in graphs]
    try:
        counts, om, ov, s, st = P.pv_count_global_batch_raw(ctx, hs, cap=8)
    finally:
        for h in hs:
            P.pv_graph_free(h)
    assert s == P.PV_EBUFSIZE
    assert st["status"] == [P.PV_OK, P.PV_EBUFSIZE, P.PV_OK, P.PV_OK]
    for i in (0, 2, 3):
        ref = O.count(graphs[i]).glob
        assert P.u128_to_ints(counts[i])[: min(8, len(ref))] == ref[:8], i


# ------------------------------------------------------- tuning cache

def test_autotune_cache_round_trip(tmp_path):
    import torch
    path = str(tmp_path / "tune.json")
    g = gg.plant_cliques(gg.chung_lu(40_000, 16, 2.3, 2000, 44), [40, 25], 45)
    ref = O.count(g, vertex=(3, 6))
    c1 = P.pv_init(0, tune_cache=path)
    dev = torch.zeros((g.n, 4, 2), dtype=torch.int64, device="cuda:0")
    try:
        h = P.pv_graph_load_csr(c1, g.n, g.row_ptr, g.col)
        t = P.pv_autotune(h, P.PV_VERTEX, 3, 6, dev.data_ptr(), reps=1)
        key = P.pv_tune_key(h, P.PV_VERTEX, 3, 6)
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c1)
    _say(f"[boundary] tuned {t} for {key}")
    assert t["trials"] >= 10 and t["ms_best"] <= t["ms_default"]
    with open(path) as f:
        entries = {e["key"]: e for e in json.load(f)["entries"]}
    assert entries[key]["dfs_max"] == t["dfs_max"] and entries[key]["lane_max"] == t["lane_max"]
    assert entries[key]["dfs_budget"] == t["dfs_budget"]
    # a new context reads the cache; the tuned walk builds the same tree
    c2 = P.pv_init(0, tune_cache=path)
    try:
        h = P.pv_graph_load_csr(c2, g.n, g.row_ptr, g.col)
        assert P.pv_tune_key(h, P.PV_VERTEX, 3, 6) == key
        dev.zero_()
        res, lov = P.pv_count(h, local_kind=P.PV_VERTEX, k_lo=3, k_hi=6, local_out=dev.data_ptr())
        torch.cuda.synchronize()
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c2)
    assert res.counts[: len(ref.glob)] == ref.glob and lov == 0
    assert res.stats["leaves"] == ref.stats["leaves"] and res.stats["nodes"] == ref.stats["nodes"]
    assert np.array_equal(dev.cpu().numpy().view(np.uint64), ref.vertex)


# --------------------------------------------- local counts of root subsets

@pytest.mark.parametrize("kind", [P.PV_VERTEX, P.PV_EDGE])
def test_root_subset_local_counts(ctx, kind):
    import torch
    g = gg.plant_cliques(gg.chung_lu(5000, 14, 2.4, 400, 46), [70, 30], 47)
    with_h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    try:
        sub = P.pv_graph_export_order(with_h)
        od = O.out_degrees(g, sub)
        rng = np.random.default_rng(48)
        roots = np.concatenate([rng.choice(np.nonzero(od > 0)[0], 400, replace=False),
                                np.argsort(-od)[:3], np.nonzero(od == 0)[0][:3]])
        roots = np.unique(roots).astype(np.int32)
        klo, khi = (3, 10) if kind == P.PV_VERTEX else (3, 8)
        rows = g.n if kind == P.PV_VERTEX else g.m
        dev = torch.zeros((rows, khi - klo + 1, 2), dtype=torch.int64, device="cuda:0")
        got, lov = P.pv_count_roots(with_h, roots, local_kind=kind, k_lo=klo, k_hi=khi,
                                    local_out=dev.data_ptr(), with_local_ovf=True)
        torch.cuda.synchronize()
    finally:
        P.pv_graph_free(with_h)
    kw = {"vertex": (klo, khi)} if kind == P.PV_VERTEX else {"edge": (klo, khi)}
    ref = O.count(g, key=sub, roots=roots, **kw)
    table = ref.vertex if kind == P.PV_VERTEX else ref.edge
    assert lov == 0 and od[roots].max() > 64
    assert got.counts[1: len(ref.glob)] == ref.glob[1:]
    assert np.array_equal(dev.cpu().numpy().view(np.uint64), table)


def test_measure_peaks_plausible():
    """The roofline denominators: every rate positive and below what the
    device could ever reach (published HBM 8 TB/s; VALU 2x the per-lane
    integer rate, allowing dual issue; LDS 256 CUs x 256 B per clock)."""
    ctx = P.pv_init(0)
    try:
        pk = P.pv_measure_peaks(ctx, 256 << 20)
    finally:
        P.pv_fini(ctx)
    _say(f"[boundary] measured peaks {pk}")
    assert 100.0 < pk["hbm_copy_gbs"] < 8000.0 * 1.05
    assert 100.0 < pk["hbm_read_gbs"] < 8000.0 * 1.05
    assert 1000.0 < pk["lds_read_gbs"] < 256 * 256 * 2.5
    assert 1000.0 < pk["valu_gops"] < 2 * 256 * 64 * 2.5
    assert all(pk[k] > 0 for k in ("ms_copy", "ms_read", "ms_lds", "ms_valu"))


# ------------------------------------- level buffers that do not fit at once

def test_heavy_roots_split_into_chunks_under_a_budget():
    """When the level buffers of all heavy roots at once do not fit the
    budget, the walk halves the heavy-root chunk and starts over: same
    counts, more chunks, never above the budget."""
    g = gg.rmat_web(scale=13)
    c0 = P.pv_init(0)
    try:
        h = P.pv_graph_load_csr(c0, g.n, g.row_ptr, g.col)
        ref = P.pv_count_global(h, 8)
        held = P.pv_memory(c0)
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c0)
    _say(f"[boundary] rmat13 k<=8: {ref.stats['heavy_chunks']} chunk(s), {held} bytes held, "
         f"nodes {ref.stats['nodes']}")
    assert ref.stats["heavy_chunks"] == 1
    seen = []
    for frac in (0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3):
        budget = int(held * frac)
        c = P.pv_init(0, hbm_budget=budget)
        try:
            h = P.pv_graph_load_csr(c, g.n, g.row_ptr, g.col)
            try:
                res = P.pv_count_global(h, 8)
            except P.PivoterError as e:
                assert e.status == P.PV_ENOMEM
                res = None
            assert P.pv_memory(c) <= budget
            P.pv_graph_free(h)
        finally:
            P.pv_fini(c)
        if res is None:
            break
        assert res.counts == ref.counts and res.omega == ref.omega
        assert res.stats["leaves"] == ref.stats["leaves"]
        seen.append((frac, res.stats["heavy_chunks"]))
    _say(f"[boundary] budget fraction -> heavy chunks: {seen}")
    assert any(ch > 1 for _, ch in seen), seen


# ------------------------------------------- cancellation and the watchdog

@pytest.fixture(scope="module")
def long_call_graph():
    # per-edge counts of k = 3..8 on an R-MAT graph of 2^14 vertices: a call
    # of about a second
    return gg.rmat_web(scale=14)


def _timed_edge_count(h):
    t0 = time.perf_counter()
    try:
        P.pv_count_local(h, P.PV_EDGE, 3, 8)
        st = P.PV_OK
    except P.PivoterError as e:
        st = e.status
    return st, time.perf_counter() - t0


def test_cancel_stops_a_running_call_and_the_context_stays_usable(long_call_graph):
    g = long_call_graph
    c = P.pv_init(0)
    try:
        h = P.pv_graph_load_csr(c, g.n, g.row_ptr, g.col)
        ref = P.pv_count_global(h, 3)
        # a cancellation while nothing runs does not touch the next call
        P.pv_cancel(c)
        assert P.pv_count_global(h, 3).counts == ref.counts
        st, t_full = _timed_edge_count(h)
        assert st == P.PV_OK
        out = {}

        def run():
            out["status"], out["s"] = _timed_edge_count(h)

        t = threading.Thread(target=run)
        t.start()
        time.sleep(0.15 * t_full)
        P.pv_cancel(c)
        t.join()
        _say(f"[boundary] full call {t_full:.3f} s, cancelled at {0.15 * t_full:.3f} s, "
             f"returned after {out['s']:.3f} s")
        assert out["status"] == P.PV_ECANCELLED
        assert out["s"] < 0.7 * t_full
        res = P.pv_count_global(h, 3)
        assert res.counts == ref.counts and res.stats["leaves"] == ref.stats["leaves"]
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c)


def test_watchdog_stops_a_call_past_its_timeout(long_call_graph):
    g = long_call_graph
    small = gg.plant_cliques(gg.gnp(2000, 0.01, 51), [12], 52)
    c = P.pv_init(0, timeout_ms=100)
    try:
        h = P.pv_graph_load_csr(c, g.n, g.row_ptr, g.col)
        st, dt = _timed_edge_count(h)
        _say(f"[boundary] stopped by the watchdog after {dt:.3f} s")
        assert st == P.PV_ETIMEDOUT and dt < 0.8
        P.pv_graph_free(h)
        hs = P.pv_graph_load_csr(c, small.n, small.row_ptr, small.col)
        res = P.pv_count_global(hs)
        P.pv_graph_free(hs)
    finally:
        P.pv_fini(c)
    want = O.count(small).glob
    assert res.counts[: len(want)] == want


# ---------------------------------------------------------- run records

def test_run_records(tmp_path, monkeypatch):
    path = tmp_path / "runs.jsonl"
    monkeypatch.setenv("PV_RECORD", str(path))
    g = gg.plant_cliques(gg.gnp(800, 0.02, 53), [15], 54)
    c = P.pv_init(0)
    monkeypatch.delenv("PV_RECORD")
    try:
        h = P.pv_graph_load_csr(c, g.n, g.row_ptr, g.col)
        r1 = P.pv_count_global(h)
        _, _, st2 = P.pv_count_local(h, P.PV_VERTEX, 3, 6)
        P.pv_graph_free(h)
    finally:
        P.pv_fini(c)
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert [r["call"] for r in recs] == ["count", "local"]
    assert recs[0]["local"] == "none" and recs[1]["local"] == "vertex"
    assert (recs[1]["k_lo"], recs[1]["k_hi"]) == (3, 6)
    assert recs[0]["nodes"] == r1.stats["nodes"] and recs[0]["leaves"] == r1.stats["leaves"]
    assert recs[0]["omega"] == r1.omega and recs[0]["status"] == P.PV_OK
    assert recs[1]["leaves"] == st2["leaves"] and recs[0]["n"] == g.n and recs[0]["m"] == g.m
