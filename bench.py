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
  serve  an open-loop Poisson stream (200 requests/s) over a pool of 256
         Chung-Lu graphs (edge counts log-uniform in [1e3, 2e6], exponent
         2.5); graph per request Zipf(1.1) over the pool, type 50/50 global
         all-k / global + per-vertex k=3..8.  The library's serving loop with
         batching against the same loop taking one request per pass;
         latency from the scheduled arrival to the result in host memory.

The roofline object describes the dominant kernel (the compact-item
specialisation of the SCT level kernel): integer ALU work, its launches
timed with HIP events on the library's stream, and its HBM traffic from
counter runs while the kernel sources are unchanged.  The cpu_baseline
object times the CPU oracle (single thread) on a stratified sample of root
subproblems and scales each stratum by its exact SCT node count.
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
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one 32-bit integer
# operation per lane per clock on the vector ALUs
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
K_LO, K_HI = 3, 10
# HBM traffic of the dominant kernel from two rocprofv3 counter runs
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


def measured_traffic(kernel: str):
    """Bytes per launch of `kernel` from the committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash() or t.get("kernel") != kernel:
        return None
    return t.get("hbm_bytes_per_launch")


def make_graph():
    from paper_2001_06784_amd import graphgen as gg
    return gg.chung_lu_social(n=1_000_000, avg_deg=20.0, gamma=2.3, max_deg=20_000.0, seed=1)


def cpu_baseline(g, h, total_nodes: int, seed: int, heavy_sample: int = 16,
                 light_fraction: float = 0.02):
    """The oracle as it stands, single-threaded: its own peel over the whole
    graph plus the SCT and Alg. 2 updates (global all k, per-vertex
    k=3..10) for a sample of roots, scaled to the whole graph.

    Root subproblems are independent (Sec. 5) but their costs are extremely
    skewed, so the scaling is a ratio estimate per stratum: the oracle's
    time per SCT node on sampled roots times the stratum's exact node count.
    Strata: roots with |N+(v)| > 62 and the others; their node counts come
    from the GPU (the same tree: node counts are parity-tested), the heavy
    stratum from one pv_count_roots call, the rest as the remainder of the
    timed run's total."""
    from oracle import oracle as O
    from paper_2001_06784_amd import pivoter as P
    t0 = time.perf_counter()
    pe = O.peel(g)
    t_peel = time.perf_counter() - t0
    od = O.out_degrees(g, pe.sub)
    rng = np.random.default_rng(seed)
    heavy = np.nonzero(od > 62)[0].astype(np.int32)
    light = np.nonzero((od > 0) & (od <= 62))[0].astype(np.int32)
    sinks = int(np.sum(od == 0))
    nh = min(heavy_sample, len(heavy))
    nl = max(1, int(round(light_fraction * len(light))))
    hs = np.sort(rng.choice(heavy, nh, replace=False)).astype(np.int32) if nh else heavy[:0]
    ls = np.sort(rng.choice(light, nl, replace=False)).astype(np.int32)
    N_h = P.pv_count_roots(h, heavy).stats["nodes"] if len(heavy) else 0
    N_l = total_nodes - N_h - sinks
    t_h = n_h = 0
    if nh:
        t0 = time.perf_counter()
        rh = O.count(g, key=pe.sub, roots=hs, vertex=(K_LO, K_HI))
        t_h = time.perf_counter() - t0
        n_h = rh.stats["nodes"]
    t0 = time.perf_counter()
    rl = O.count(g, key=pe.sub, roots=ls, vertex=(K_LO, K_HI))
    t_l = time.perf_counter() - t0
    n_l = rl.stats["nodes"]
    t_full = t_peel + (t_h * N_h / n_h if n_h else 0.0) + (t_l * N_l / n_l if n_l else 0.0)
    return {
        "value": g.m / t_full,
        "unit": "edges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{nh} of {len(heavy)} roots with |N+(v)| > 62 ({t_h:.1f} s, {n_h} SCT nodes) "
                   f"and {nl} of {len(light)} others ({t_l:.1f} s, {n_l} nodes), seed {seed}; "
                   f"global all-k + per-vertex k={K_LO}..{K_HI}; each stratum's seconds per node "
                   f"times its exact node count ({N_h} and {N_l}), plus the full peel "
                   f"{t_peel:.2f} s; estimated full run {t_full:.0f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["social", "batch", "serve", "copy", "rmat"], default="social")
    ap.add_argument("--scale", type=int, default=14, help="rmat: log2 of the vertex count")
    ap.add_argument("--edge", action="store_true", help="rmat: also per-edge counts for k=3..8")
    ap.add_argument("--duration", type=float, default=20.0, help="serve: measured seconds")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the roots over "
              "several GPUs is not built", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "copy":
        return bench_copy()
    if args.workload == "rmat":
        return bench_rmat(args)

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
    levels = sum(s["levels"] for s in stats)
    ms_levels = sum(s["ms_levels"] for s in stats)
    # the level kernel is specialised per unit kind; the dominant kernel is
    # the specialisation with the largest summed device time
    kinds = ("multi-word", "compact-items", "light-roots")
    ms_kind = [sum(s["ms_kind"][i] for s in stats) for i in range(3)]
    launches = [sum(s["launches_kind"][i] for s in stats) for i in range(3)]
    work = [sum(s["work_kind"][i] for s in stats) for i in range(3)]
    dom = max(range(3), key=lambda i: ms_kind[i])
    # algorithmic ALU work: each 64-bit AND + popcount of the pivot search is
    # 4 lane operations (two 32-bit ANDs, two 32-bit bit counts)
    achieved_tops = 4.0 * work[dom] / (ms_kind[dom] * 1e-3) / 1e12 if ms_kind[dom] > 0 else 0.0
    kname = f"sct_level_kernel<{st['kernel_kl']}, {dom}, {st['kernel_lk']}>"
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
        "roofline": {
            "bound": "alu",
            "kernel": f"{kname} ({kinds[dom]})",
            "achieved": achieved_tops,
            "peak": ALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved_tops / ALU_PEAK_TOPS,
            "traffic": measured_traffic(kname),
            "avg_launch_ms": ms_kind[dom] / max(launches[dom], 1),
            "launches": launches[dom],
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, h, st["nodes"], seed=7)
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
    ctx = P.pv_init(0, torch.cuda.current_stream().cuda_stream)
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    for i in range(max(1, args.warmup)):
        t1 = time.perf_counter()
        P.pv_count_global(h)
        print(f"[bench] warm-up {i}: {time.perf_counter() - t1:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = P.pv_count_global(h)
        print(f"[bench] step {i}: {time.perf_counter() - t0:.2f} s so far", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = res.stats
    line = {
        "metric": "graph edges/sec and SCT leaves/sec for all-k counts", "value": g.m / dt, "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup), "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u128",
        "data": "synthetic", "leaves_per_s": st["leaves"] / dt,
        "config": {"workload": (f"rmat scale={args.scale} edge_factor=24 a=0.57 b=0.19 c=0.19 seed=1 "
                                "+ 50 planted cliques of 20..60; global counts all k"),
                   "n": g.n, "m": g.m, "alpha": st["alpha"], "omega": res.omega,
                   "sct_nodes": st["nodes"], "sct_leaves": st["leaves"], "overflow_k": res.overflow},
    }
    if args.edge:
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
