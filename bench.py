#!/usr/bin/env python
"""Benchmark of the exact clique-counting hot path on one MI355X.

Workload: a heavy-tailed Chung-Lu graph (n = 1,000,000, average degree 20,
degree exponent 2.3, expected degrees capped at 20,000, seed 1; about 9.9M
edges), standing in for the paper's social networks.  One step is the whole
path on a device-resident CSR: degeneracy orientation, Succinct Clique Tree,
global counts for every k, and per-vertex counts for k = 3..10, all in one
pv_count call.

Prints one JSON line.  value = undirected edges / second of wall time per
step; leaves_per_s = SCT leaves / second.

Other workloads are selected with --workload:
  batch  4096 small Chung-Lu graphs (n log-uniform in [50, 5000], average
         degree uniform in [8, 40], exponent 2.5), global counts for all k:
         one batched union pass against one call per graph (graphs/s).
  rmat   global counts for all k on an R-MAT graph (--scale, edge factor 24,
         a/b/c = 0.57/0.19/0.19) with 50 planted cliques of 20..60 vertices;
         --edge adds per-edge counts for k = 3..8.  Scale 22 itself is a
         parity case: its tree is far too large to walk whole.
  serve  (disabled: see main) an open-loop Poisson stream (200 requests/s) over a pool of 256
         Chung-Lu graphs (edge counts log-uniform in [1e3, 2e6], exponent
         2.5); graph per request Zipf(1.1) over the pool, type 50/50 global
         all-k / global + per-vertex k=3..8.  The library's serving loop with
         batching against the same loop taking one request per pass;
         latency from the scheduled arrival to the result in host memory.

The roofline object describes the dominant kernel, the SCT level kernel
(every unit kind): its algorithmic VALU, LDS and HBM work per launch (the
model is stated with the constants below), each against MI355X's published
or derived peak and against the rates pv_measure_peaks measures on this
device, over its launches' summed durations (HIP events on each launch's
stream), and its HBM traffic from counter runs while the kernel sources are
unchanged.  The cpu_baseline
object times the CPU oracle in the paper's parallel form (independent root
subproblems over worker processes on the host's cores) on a systematic
sample of every 16th root by out-degree rank, scaled by 16.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "graph edges/sec and SCT leaves/sec for all-k counts; p50/p99 request latency"
# MI355X published/derived peaks: HBM3E 8 TB/s; 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz = one 32-bit integer operation per lane per clock on the vector
# ALUs; LDS 128 bytes per clock per CU
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
LDS_PEAK_GBS = 256 * 128 * 2.4e9 / 1e9
K_LO, K_HI = 3, 10
# The level kernel's algorithmic work per unit (the roofline model):
#   VALU lane operations: 4 per 64-bit AND + popcount pair of the pivot
#   search (two ANDs, two bit counts), 2 per word of a child's vertex set
#   (one 64-bit AND), 2 per per-vertex addition of Alg. 2 (a 64-bit add),
#   of which there are K per leaf vertex: sum over leaves of (h + p) * K;
#   LDS bytes: a child's set word is written to the on-chip stack and read
#   back (16); the per-vertex sums stay in registers and a leaf's binomial
#   rows come through the scalar cache, so the additions add no LDS bytes;
#   HBM bytes: the compulsory ones, every root's gather of N+(v) and its
#   members' N+(u) (4 per id, 8 per row-pointer pair) and the per-vertex
#   table written once (16 per u128 count).
VALU_PER_PAIR, VALU_PER_CHILD_WORD, VALU_PER_ADD = 4, 2, 2
LDS_PER_CHILD_WORD = 16
# HBM traffic of the level kernel from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE), each scaled by what the same counter reads for a
# plain copy of known size; valid only for the kernel sources it was taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sct_level_kernel_chunglu1M_vertex3-10.json")
KERNEL_SOURCES = ["paper_2001_06784_amd/csrc/sct.hip", "paper_2001_06784_amd/csrc/common.h",
                  "paper_2001_06784_amd/csrc/internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per step of the level kernel (all its launches) from the
    committed counter summary, or None when it is missing or was taken on
    other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_step")


def compulsory_hbm_bytes(g, key, K):
    """The level kernel's compulsory HBM bytes for one step: the gathers of
    every root (N+(v), then N+(u) of each member u) and the per-vertex
    table written once.  Edge a->b iff (key[a], a) < (key[b], b)."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    cols = g.col.astype(np.int64)
    fwd = (key[rows] < key[cols]) | ((key[rows] == key[cols]) & (rows < cols))
    od = np.bincount(rows[fwd], minlength=g.n).astype(np.int64)
    ind = deg - od
    gathers = 8 * g.n + 4 * int(od.sum()) + int((ind * (8 + 4 * od)).sum())
    return gathers + 16 * g.n * K


def roofline(stats, peaks, hbm_bytes, traffic):
    """Roofline of the SCT level kernel (every unit kind) over the timed
    steps: each term's algorithmic units over its peak, against the summed
    launch durations (HIP events on each launch's stream)."""
    K = K_HI - K_LO + 1
    work = sum(s["work"] for s in stats)
    child = sum(s["child_work"] for s in stats)
    adds = K * sum(s["leaf_hp"] for s in stats)
    ms = sum(sum(s["ms_kind"]) for s in stats)
    ms_wall = sum(s["ms_levels"] for s in stats)
    launches = sum(sum(s["launches_kind"]) for s in stats)
    steps = len(stats)
    units = {
        "valu": VALU_PER_PAIR * work + VALU_PER_CHILD_WORD * child + VALU_PER_ADD * adds,
        "lds": LDS_PER_CHILD_WORD * child,
        "hbm": hbm_bytes * steps,
    }
    peak = {"valu": ALU_PEAK_TOPS * 1e12, "lds": LDS_PEAK_GBS * 1e9, "hbm": HBM_PEAK_GBS * 1e9}
    meas = {"valu": peaks["valu_gops"] * 1e9, "lds": peaks["lds_read_gbs"] * 1e9,
            "hbm": peaks["hbm_copy_gbs"] * 1e9}
    terms = {}
    for t in ("valu", "lds", "hbm"):
        terms[t] = {"units_per_launch": units[t] / max(launches, 1),
                    "t_ms_at_peak": units[t] / peak[t] * 1e3 / max(launches, 1),
                    "frac": units[t] / peak[t] * 1e3 / ms if ms > 0 else 0.0,
                    "peak_measured": meas[t] / (1e12 if t == "valu" else 1e9),
                    "frac_measured": units[t] / meas[t] * 1e3 / ms if ms > 0 and meas[t] > 0 else 0.0}
    bound = max(terms, key=lambda t: units[t] / peak[t])
    scale, unit = {"valu": (1e12, "TOP/s"), "lds": (1e9, "GB/s"), "hbm": (1e9, "GB/s")}[bound]
    achieved = units[bound] / (ms * 1e-3) / scale if ms > 0 else 0.0
    return {
        "bound": {"valu": "alu", "lds": "lds", "hbm": "hbm"}[bound],
        "kernel": "sct_level_kernel (every unit kind)",
        "achieved": achieved,
        "peak": peak[bound] / scale,
        "unit": unit,
        "frac": achieved * scale / peak[bound],
        "traffic": (traffic / max(launches / steps, 1)) if traffic is not None else None,
        "avg_launch_ms": ms / max(launches, 1),
        "launches": launches,
        "terms": terms,
        "frac_wall": units[bound] / peak[bound] * 1e3 / ms_wall if ms_wall > 0 else 0.0,
        "work_per_step": {"pivot_pairs": work / steps, "child_words": child / steps,
                          "vertex_additions": adds / steps, "compulsory_hbm_bytes": hbm_bytes},
        "peaks_measured": peaks,
    }


def make_graph():
    from paper_2001_06784_amd import graphgen as gg
    return gg.chung_lu_social(n=1_000_000, avg_deg=20.0, gamma=2.3, max_deg=20_000.0, seed=1)


def _cpu_info():
    """(nproc, CPU model name) of this host, as lscpu reports them."""
    import subprocess
    nproc = os.cpu_count()
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return nproc, model


def cpu_baseline(g, stride: int = 16, max_workers: int = 16):
    """The oracle as it stands, in the paper's parallel form (Sec. 5: the
    root subproblems are independent; workers count them with private
    counters and the counts are summed), on the host cores this process
    may use (at most max_workers): its own peel over the whole graph, then
    the SCT and Alg. 2 updates (global all k, per-vertex k=3..10) for a
    systematic sample of the roots -- every `stride`-th root in order of
    out-degree, so the sample holds the same share of every degree rank --
    whose wall time times `stride` stands for the whole graph.  Nothing in
    it comes from the GPU."""
    from oracle import oracle as O
    from oracle import parallel as OP
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    pe = O.peel(g)
    t_peel = time.perf_counter() - t0
    od = O.out_degrees(g, pe.sub)
    order = np.argsort(-od, kind="stable").astype(np.int32)
    sample = np.sort(order[::stride])
    t0 = time.perf_counter()
    r = OP.count_parallel(g, pe.sub, roots=sample, workers=workers, vertex=(K_LO, K_HI))
    t_sample = time.perf_counter() - t0
    t_full = t_peel + stride * t_sample
    nproc, model = _cpu_info()
    return {
        "value": g.m / t_full,
        "unit": "edges/s",
        "cores": r["workers"],
        "kind": "oracle",
        "sample": (f"every {stride}th root by out-degree rank ({len(sample)} of {g.n} roots, "
                   f"{r['stats']['nodes']} SCT nodes), global all-k + per-vertex k={K_LO}..{K_HI}, "
                   f"oracle in the paper's parallel form on {r['workers']} processes: {t_sample:.1f} s wall "
                   f"({r['busy_s']:.1f} s busy summed); the full peel {t_peel:.2f} s; estimated whole graph "
                   f"{t_full:.0f} s = peel + {stride} x sample; host nproc {nproc}, {model}"),
        "nproc": nproc,
        "cpu": model,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["social", "batch", "serve", "copy", "rmat"], default="social")
    ap.add_argument("--scale", type=int, default=14, help="rmat: log2 of the vertex count")
    ap.add_argument("--edge", action=argparse.BooleanOptionalAction, default=None,
                    help="also per-edge counts for k=3..8 (one warm-up call, one timed call; not in the step); "
                         "default: on for the social workload, off for rmat")
    ap.add_argument("--kmax", type=int, default=0, help="rmat: global counts truncated at k <= kmax (0: all k)")
    ap.add_argument("--sample", action="store_true",
                    help="rmat: time the root subtrees of a stratified root sample instead of the whole graph")
    ap.add_argument("--sample-scale", type=int, default=20,
                    help="rmat --sample: roots per stratum as a multiple of the parity tests' sample (1: that sample)")
    ap.add_argument("--duration", type=float, default=20.0, help="serve: measured seconds")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the roots over "
              "several GPUs is not built", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        # Off until its GPU memory fault is explained: two runs of this
        # workload (each after runs of the test suite in the same session)
        # ended with the device faulted, and no cause has been found in the
        # serving loop or the kernels it launches.  The serving tests, with
        # small graphs, pass.
        print("bench.py --workload serve is disabled: it has ended with a GPU memory fault whose cause "
              "is not found", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        return bench_copy()
    if args.workload == "rmat":
        args.edge = bool(args.edge)
        return bench_rmat(args)
    args.edge = args.edge is None or args.edge

    import torch
    from paper_2001_06784_amd import pivoter as P

    t0 = time.perf_counter()
    g = make_graph()
    print(f"[bench] graph n={g.n} m={g.m} generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    ctx = P.pv_init(0, torch.cuda.current_stream().cuda_stream)
    P.pv_set_timing(ctx, True)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    K = K_HI - K_LO + 1
    local = torch.zeros((g.n, K, 2), dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    peaks = P.pv_measure_peaks(ctx)
    print(f"[bench] measured peaks: {peaks}", file=sys.stderr, flush=True)

    def step():
        res, lovf = P.pv_count(h, reorient=True, local_kind=P.PV_VERTEX, k_lo=K_LO, k_hi=K_HI,
                               local_out=local.data_ptr())
        assert lovf == 0 and res.status == P.PV_OK
        return res

    for i in range(args.warmup):
        res = step()
        print(f"[bench] warmup {i}: omega={res.omega} leaves={res.stats['leaves']}",
              file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        res = step()
        stats.append(res.stats)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    print(f"[bench] {args.steps} steps, {dt * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    st = stats[-1]
    kinds = ("multi-word", "compact-items", "light-roots")
    key = P.pv_graph_export_order(h)
    roof = roofline(stats, peaks, compulsory_hbm_bytes(g, key, K), measured_traffic())
    line = {
        "metric": METRIC,
        "value": g.m / dt,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u128",
        "data": "synthetic",
        "leaves_per_s": st["leaves"] / dt,
        "config": {
            "workload": ("chung-lu n=1000000 avg_deg=20 gamma=2.3 max_deg=20000 seed=1; "
                         f"global counts all k + per-vertex k={K_LO}..{K_HI}"),
            "n": g.n, "m": g.m, "alpha": st["alpha"], "omega": st["omega"],
            "sct_nodes": st["nodes"], "sct_leaves": st["leaves"], "parallelism": "1 GPU",
        },
        "device_ms": {"peel": st["ms_peel"], "orient": st["ms_orient"],
                      "levels": st["ms_levels"], "finalize": st["ms_finalize"],
                      "level_launches": st["levels"],
                      "levels_by_kind": {kinds[i]: st["ms_kind"][i] for i in range(3)}},
        "roofline": roof,
    }
    if args.edge:
        # per-edge counts for k = 3..8 into a device table (m x 6 u128), after
        # the timed steps; the graph is already oriented and the tree is cut at
        # k_max = 8 hold vertices (Sec. 5, counting for a specific k)
        del local
        eloc = torch.zeros((g.m, 6, 2), dtype=torch.int64, device="cuda:0")
        P.pv_count(h, reorient=False, k_max=8, local_kind=P.PV_EDGE, k_lo=3, k_hi=8, local_out=eloc.data_ptr())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        eres, eovf = P.pv_count(h, reorient=False, k_max=8, local_kind=P.PV_EDGE, k_lo=3, k_hi=8,
                                local_out=eloc.data_ptr())
        torch.cuda.synchronize()
        te = time.perf_counter() - t1
        est = eres.stats
        line["per_edge_k3_8"] = {"s": te, "edges_per_s": g.m / te, "overflow": int(eovf),
                                 "sct_nodes": est["nodes"], "sct_leaves": est["leaves"],
                                 "device_ms": {"levels": est["ms_levels"],
                                               "levels_by_kind": {kinds[i]: est["ms_kind"][i] for i in range(3)}}}
        print(f"[bench] per-edge k=3..8: {te:.3f} s", file=sys.stderr, flush=True)
        del eloc
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g)
    P.pv_graph_free(h)
    P.pv_fini(ctx)
    print(json.dumps(line), flush=True)


def bench_batch(args):
    import torch
    from paper_2001_06784_amd import graphgen as gg
    from paper_2001_06784_amd import pivoter as P
    t0 = time.perf_counter()
    graphs = gg.batch_graphs()
    print(f"[bench] {len(graphs)} graphs generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    ctx = P.pv_init(0, torch.cuda.current_stream().cuda_stream)
    hs = [P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col) for g in graphs]
    m_total = sum(g.m for g in graphs)
    for _ in range(args.warmup):
        P.pv_count_global_batch_raw(ctx, hs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts, om, ov, s, st = P.pv_count_global_batch_raw(ctx, hs)
    dt = (time.perf_counter() - t0) / args.steps
    # the plain path: one pv_count_global call per graph, same GPU
    lat = []
    t1 = time.perf_counter()
    for h in hs:
        t2 = time.perf_counter()
        P.pv_count_global(h)
        lat.append(time.perf_counter() - t2)
    dt_plain = time.perf_counter() - t1
    for h in hs:
        P.pv_graph_free(h)
    P.pv_fini(ctx)
    line = {
        "metric": "graphs/sec, batched global all-k counts", "value": len(hs) / dt, "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u128",
        "data": "synthetic",
        "config": {"workload": "4096 Chung-Lu graphs, n log-uniform [50,5000], avg deg U[8,40], "
                               "gamma 2.5, seeds 1000+i; global counts all k",
                   "graphs": len(hs), "m_total": m_total, "sct_leaves": st["leaves"]},
        "edges_per_s": m_total / dt,
        "plain": {"graphs_per_s": len(hs) / dt_plain, "s": dt_plain,
                  "p50_ms_per_graph": 1e3 * float(np.percentile(lat, 50)),
                  "p99_ms_per_graph": 1e3 * float(np.percentile(lat, 99))},
        "batched_over_plain": (len(hs) / dt) / (len(hs) / dt_plain),
    }
    print(json.dumps(line), flush=True)


def bench_rmat(args):
    """Whole-graph global counts for all k on an R-MAT graph with 50 planted
    cliques (the web-like workload at a scale small enough to finish); the
    warm-up call also sizes the work buffers, so timed calls walk the tree
    once.  With --edge, per-edge counts for k = 3..8 as well."""
    import torch
    from paper_2001_06784_amd import graphgen as gg
    from paper_2001_06784_amd import pivoter as P
    t0 = time.perf_counter()
    g = gg.rmat_web(scale=args.scale)
    print(f"[bench] rmat scale {args.scale}: n={g.n} m={g.m} generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    # a sampled-root run stops with PV_ETIMEDOUT rather than run on if a
    # call takes more than two minutes
    ctx = P.pv_init(0, torch.cuda.current_stream().cuda_stream, timeout_ms=120000 if args.sample else 0)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    if args.sample:
        return bench_rmat_sample(args, g, ctx, h)
    for i in range(max(1, args.warmup)):
        t1 = time.perf_counter()
        P.pv_count_global(h, args.kmax)
        print(f"[bench] warm-up {i}: {time.perf_counter() - t1:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = P.pv_count_global(h, args.kmax)
        print(f"[bench] step {i}: {time.perf_counter() - t0:.2f} s so far", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = res.stats
    line = {
        "metric": ("graph edges/sec and SCT leaves/sec for all-k counts" if not args.kmax else
                   f"graph edges/sec for counts of k <= {args.kmax} (tree truncated at k_max)"),
        "value": g.m / dt, "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup), "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u128",
        "data": "synthetic", "leaves_per_s": st["leaves"] / dt,
        "config": {"workload": (f"rmat scale={args.scale} edge_factor=24 a=0.57 b=0.19 c=0.19 seed=1 "
                                "+ 50 planted cliques of 20..60; global counts "
                                + (f"k <= {args.kmax}" if args.kmax else "all k")),
                   "n": g.n, "m": g.m, "alpha": st["alpha"], "omega": res.omega,
                   "sct_nodes": st["nodes"], "sct_leaves": st["leaves"], "overflow_k": res.overflow},
    }
    if args.edge:
        if args.warmup > 0:
            P.pv_count_local(h, P.PV_EDGE, 3, 8)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out, ovf, est = P.pv_count_local(h, P.PV_EDGE, 3, 8)
        torch.cuda.synchronize()
        te = time.perf_counter() - t1
        # the call returns the m x 6 u128 counts in host memory (copy included)
        line["per_edge_k3_8"] = {"s": te, "edges_per_s": g.m / te, "overflow": int(ovf),
                                 "sct_nodes": est["nodes"], "sct_leaves": est["leaves"]}
    P.pv_graph_free(h)
    P.pv_fini(ctx)
    print(json.dumps(line), flush=True)


def rmat_root_sample(g, key, scale=1):
    """A seeded sample of roots in out-degree strata (0, 64], (64, 128],
    (128, 256], (256, 512] (scale x 2000, 40, 10 and 5 roots) plus 5 roots
    of out-degree 0.  With scale 1 it is the sample the sampled-root parity
    tests check against the oracle.  Edge a->b iff (key[a], a) < (key[b], b)."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    cols = g.col.astype(np.int64)
    fwd = (key[rows] < key[cols]) | ((key[rows] == key[cols]) & (rows < cols))
    od = np.bincount(rows[fwd], minlength=g.n)
    rng = np.random.default_rng(2022)
    parts = []
    for lo, hi, cnt in [(0, 64, 2000), (64, 128, 40), (128, 256, 10), (256, 512, 5)]:
        pool = np.nonzero((od > lo) & (od <= hi))[0]
        parts.append(rng.choice(pool, min(cnt * scale, len(pool)), replace=False))
    parts.append(np.nonzero(od == 0)[0][:5])
    return np.concatenate(parts).astype(np.int32), od


def bench_rmat_sample(args, g, ctx, h):
    """SCT leaves/s of the root subtrees of a stratified root sample (the
    R-MAT protocol where the whole tree cannot be walked): global counts of
    the cliques whose smallest-key vertex is a sampled root, for all k or
    truncated at --kmax."""
    import torch
    from paper_2001_06784_amd import pivoter as P
    P.pv_graph_orient(h)
    key = P.pv_graph_export_order(h)
    roots, od = rmat_root_sample(g, key, args.sample_scale)
    print(f"[bench] {len(roots)} sampled roots, out-degrees up to {int(od[roots].max())}", file=sys.stderr, flush=True)
    for i in range(max(1, args.warmup)):
        t1 = time.perf_counter()
        P.pv_count_roots(h, roots, k_max=args.kmax)
        print(f"[bench] warm-up {i}: {time.perf_counter() - t1:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = P.pv_count_roots(h, roots, k_max=args.kmax)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = res.stats
    line = {
        "metric": "SCT leaves/sec over a stratified root sample" + (f" (k <= {args.kmax})" if args.kmax else " (all k)"),
        "value": st["leaves"] / dt, "unit": "leaves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup), "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u128", "data": "synthetic",
        "config": {"workload": (f"rmat scale={args.scale} edge_factor=24 a=0.57 b=0.19 c=0.19 seed=1 "
                                "+ 50 planted cliques of 20..60; root subtrees of a seeded sample in out-degree "
                                f"strata (0,64]:{2000 * args.sample_scale} (64,128]:{40 * args.sample_scale} "
                                f"(128,256]:{10 * args.sample_scale} (256,512]:{5 * args.sample_scale}, "
                                "5 of out-degree 0"),
                   "n": g.n, "m": g.m, "alpha": int(od.max()), "roots": int(len(roots)),
                   "max_root_out_degree": int(od[roots].max()), "omega": res.omega,
                   "sct_nodes": st["nodes"], "sct_leaves": st["leaves"], "overflow_k": res.overflow},
    }
    P.pv_graph_free(h)
    P.pv_fini(ctx)
    print(json.dumps(line), flush=True)


def bench_copy():
    """A plain device copy of 1 GiB: the known-size reference that scales the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_read": src.numel() * 4,
                      "bytes_written": dst.numel() * 4}), flush=True)


def _serve_trace(duration: float, warm: float, rate: float = 200.0):
    from paper_2001_06784_amd import graphgen as gg
    specs = gg.serve_pool_specs()
    t0 = time.perf_counter()
    pool = [gg.chung_lu(n, d, 2.5, n - 1, s) for (n, d, s) in specs]
    print(f"[bench] serving pool of {len(pool)} graphs (sum m {sum(g.m for g in pool)}) in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    arr = gg.poisson_arrivals(rate, warm + duration, seed=3)
    rng = np.random.default_rng(4)
    ranks = np.arange(1, len(pool) + 1, dtype=np.float64)
    pz = ranks ** -1.1
    pz /= pz.sum()
    perm = rng.permutation(len(pool))
    which = perm[rng.choice(len(pool), size=len(arr), p=pz)]
    kinds = rng.random(len(arr)) < 0.5
    return pool, arr, which, kinds


def _run_trace(P, pool, arr, which, kinds, warm, workers, max_batch):
    import threading
    srv = P.Server(workers=workers, max_batch=max_batch, cache_bytes=16 << 30, batch_bytes=8 << 30)
    out = [None] * len(arr)
    sub = []
    done = threading.Event()

    def waiter():
        i = 0
        while i < len(arr):
            while i >= len(sub):
                time.sleep(0.0005)
            tk, t_sched, t_sub = sub[i]
            r, counts, v = srv.wait(tk)
            out[i] = (t_sched, (t_sub - t_sched) + r.total_us * 1e-6, r.status, r.batch_size)
            i += 1
        done.set()

    th = threading.Thread(target=waiter)
    th.start()
    t_start = time.perf_counter()
    for i, t in enumerate(arr):
        now = time.perf_counter() - t_start
        if t > now:
            time.sleep(t - now)
        g = pool[which[i]]
        kind = P.PV_REQ_VERTEX if kinds[i] else P.PV_REQ_GLOBAL
        tk = srv.submit(int(which[i]), g, kind, 3, 8)
        sub.append((tk, float(t), time.perf_counter() - t_start))
    th.join()
    t_end = time.perf_counter() - t_start
    srv.stop()
    meas = [o for o in out if o[0] >= warm]
    lat = np.array([o[1] for o in meas])
    ok = all(o[2] == P.PV_OK for o in out)
    m_meas = sum(pool[which[i]].m for i in range(len(arr)) if arr[i] >= warm)
    span = max(t_end, arr[-1]) - warm
    return {"requests": len(meas), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "mean_ms": 1e3 * float(lat.mean()),
            "graphs_per_s": len(meas) / span, "edges_per_s": m_meas / span, "all_ok": ok,
            "mean_batch": float(np.mean([o[3] for o in meas])), "workers": workers,
            "max_batch": max_batch, "finished_s_after_last_arrival": t_end - float(arr[-1])}


def bench_serve(args):
    from paper_2001_06784_amd import pivoter as P
    warm = 5.0
    pool, arr, which, kinds = _serve_trace(args.duration, warm)
    P.load_library()
    served = _run_trace(P, pool, arr, which, kinds, warm, workers=2, max_batch=64)
    print(f"[bench] served: {served}", file=sys.stderr, flush=True)
    plain = _run_trace(P, pool, arr, which, kinds, warm, workers=1, max_batch=1)
    print(f"[bench] plain: {plain}", file=sys.stderr, flush=True)
    line = {
        "metric": "p50/p99 request latency (ms) and graphs/sec under a 200 req/s Poisson stream",
        "value": served["p99_ms"], "unit": "ms (p99)", "n_gpus": 1, "steps": len(arr),
        "warmup": int(np.sum(arr < warm)), "ms_per_step": served["mean_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u128",
        "data": "synthetic",
        "config": {"workload": "Poisson 200/s over 256 Chung-Lu graphs, m log-uniform [1e3,2e6], "
                               "avg deg U[8,40], gamma 2.5, Zipf(1.1) reuse, 50/50 global all-k / "
                               "global + per-vertex k=3..8", "measured_s": args.duration,
                   "warmup_s": warm},
        "served": served, "plain_one_request_per_pass": plain,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
