"""TEST INFRASTRUCTURE ONLY: the oracle in the paper's parallel form.

Sec. 5 ("Parallel version of Pivoter"): the root's children N+(v) are
independent subproblems, so a set of workers can take them in any split,
each counting with private counters, and the counts are summed at the end.
This module does exactly that around oracle.count (nothing of the method's
arithmetic is changed or re-implemented here): worker processes pull chunks
of roots from a shared cursor, add each chunk's exact counts to their own
totals, and the parent adds the workers' totals.  Only the test suite, the
stored-value scripts under tests/golden/ and the benchmark's CPU-baseline leg
use it.

Workers are started with the "spawn" method: each is a fresh interpreter that
never touches a GPU, whatever its parent did before.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

_G = None  # (graph, key, kwargs) in a worker


def _add_limbs(acc: np.ndarray, x: np.ndarray) -> int:
    """acc += x for (..., 2) uint64 (lo, hi) limb arrays, in place; returns
    the number of entries whose sum passed 2^128."""
    lo = acc[..., 0] + x[..., 0]
    carry = (lo < acc[..., 0]).astype(np.uint64)
    hi = acc[..., 1] + x[..., 1]
    ovf = int(np.count_nonzero(hi < acc[..., 1]))
    hi2 = hi + carry
    ovf += int(np.count_nonzero(hi2 < hi))
    acc[..., 0] = lo
    acc[..., 1] = hi2
    return ovf


class _Graph:
    """The CSR arrays a worker needs (g.n, g.m, g.row_ptr, g.col)."""

    def __init__(self, n, m, row_ptr, col):
        self.n, self.m, self.row_ptr, self.col = n, m, row_ptr, col


def _init(n, m, rp, col, key, kw):
    global _G
    _G = (_Graph(n, m, rp, col), key, kw)


def _worker(cursor, chunks, conn):
    from oracle import oracle as O
    g, key, kw = _G
    glob, vert, edge, stats, ovf = None, None, None, {}, 0
    busy = 0.0
    while True:
        with cursor.get_lock():
            i = cursor.value
            cursor.value += 1
        if i >= len(chunks):
            break
        t0 = time.perf_counter()
        r = O.count(g, key=key, roots=chunks[i], **kw)
        busy += time.perf_counter() - t0
        gl = [int(x) for x in r.glob]
        if glob is None:
            glob = gl
        else:
            glob = [a + b for a, b in zip(glob, gl)]
        if r.vertex is not None:
            if vert is None:
                vert = r.vertex.copy()
            else:
                ovf += _add_limbs(vert, r.vertex)
            ovf += int(r.vertex_ovf.any())
        if r.edge is not None:
            if edge is None:
                edge = r.edge.copy()
            else:
                ovf += _add_limbs(edge, r.edge)
            ovf += int(r.edge_ovf.any())
        for k, v in r.stats.items():
            if k in ("alpha", "omega", "max_depth", "need_kcap"):
                stats[k] = max(stats.get(k, 0), v)
            elif k != "subrounds":
                stats[k] = stats.get(k, 0) + v
    conn.send((glob, stats, ovf, busy))
    for arr in (vert, edge):
        conn.send(None if arr is None else arr.shape)
        if arr is not None:
            conn.send_bytes(memoryview(np.ascontiguousarray(arr)).cast("B"))
    conn.close()


def count_parallel(g, key, roots=None, workers: int | None = None, chunks: int | None = None, **kw):
    """oracle.count(g, key=key, roots=roots, **kw) computed by `workers`
    processes (default: the CPUs this process may run on) over `chunks`
    chunks of roots (default 32 per worker; roots are dealt round-robin by
    decreasing out-degree, so the heavy ones spread over the chunks, and
    workers pull chunks until none is left).  Returns a dict: glob (exact
    Python ints, C_0 = 1 for the whole graph, 0 for a root subset), vertex /
    edge limb arrays (or None), stats, overflow count, workers, and busy
    seconds summed over workers."""
    from oracle import oracle as O
    key = np.ascontiguousarray(key, dtype=np.int32)
    whole = roots is None
    if whole:
        roots = np.arange(g.n, dtype=np.int32)
    roots = np.asarray(roots, dtype=np.int32)
    od = O.out_degrees(g, key)
    order = roots[np.argsort(-od[roots], kind="stable")]
    if workers is None:
        workers = len(os.sched_getaffinity(0))
    nch = max(1, min(len(order), chunks if chunks else 32 * max(1, workers)))
    chunks = [order[i::nch].copy() for i in range(nch)]
    workers = max(1, min(workers, len(chunks)))
    ctx = mp.get_context("spawn")
    cursor = ctx.Value("l", 0)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    procs, pipes = [], []
    for _ in range(workers):
        a, b = ctx.Pipe(duplex=False)
        p = ctx.Process(target=_run_worker, args=(g.n, g.m, rp, col, key, kw, cursor, chunks, b))
        p.start()
        procs.append(p)
        pipes.append(a)
    glob, vert, edge, stats, ovf, busy = None, None, None, {}, 0, 0.0
    for conn in pipes:
        gl, st, ov, bz = conn.recv()
        ovf += ov
        busy += bz
        if gl is not None:
            glob = gl if glob is None else [x + y for x, y in zip(glob, gl)]
        for k, v in st.items():
            if k in ("alpha", "omega", "max_depth", "need_kcap"):
                stats[k] = max(stats.get(k, 0), v)
            else:
                stats[k] = stats.get(k, 0) + v
        parts = []
        for _ in range(2):
            shape = conn.recv()
            parts.append(None if shape is None else
                         np.frombuffer(conn.recv_bytes(), dtype=np.uint64).reshape(shape).copy())
        if parts[0] is not None:
            if vert is None:
                vert = parts[0]
            else:
                ovf += _add_limbs(vert, parts[0])
        if parts[1] is not None:
            if edge is None:
                edge = parts[1]
            else:
                ovf += _add_limbs(edge, parts[1])
    for p in procs:
        p.join()
        if p.exitcode != 0:
            raise RuntimeError(f"oracle worker failed with exit code {p.exitcode}")
    if glob is None:
        glob = [0]
    glob[0] = 1 if whole else 0
    return {"glob": glob, "vertex": vert, "edge": edge, "stats": stats, "overflow": ovf,
            "workers": workers, "busy_s": busy}


def _run_worker(n, m, rp, col, key, kw, cursor, chunks, conn):
    _init(n, m, rp, col, key, kw)
    _worker(cursor, chunks, conn)
