"""TEST INFRASTRUCTURE ONLY: Python access to the plain CPU oracle (oracle.c).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product library never loads it, and it shares no code
with the GPU path: the two meet only in the seeded input generators.

What the oracle computes is described in oracle.c (canonical peel, depth-first
Succinct Clique Tree, Alg. 2 leaf updates, optional truncation).  Counts come
back as exact Python integers (or as (lo, hi) uint64 limb arrays for the large
local outputs).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        i32p = C.POINTER(C.c_int32)
        u64p = C.POINTER(C.c_uint64)
        u8p = C.POINTER(C.c_uint8)
        lib.orc_peel.restype = C.c_int64
        lib.orc_peel.argtypes = [C.c_int32, i32p, i32p, i32p, i32p]
        lib.orc_count.restype = C.c_int32
        lib.orc_count.argtypes = [C.c_int32, i32p, i32p, i32p, i32p, i32p, C.c_int32, C.c_int32,
                                  C.c_int32, u64p, u8p,
                                  C.c_int32, C.c_int32, u64p, u8p,
                                  C.c_int32, C.c_int32, u64p, u8p,
                                  C.c_int32, u64p, u64p]
        _lib = lib
    return _lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(t))


def limbs_to_int(a: np.ndarray):
    """(..., 2) uint64 (lo, hi) -> nested Python ints (object array)."""
    a = np.asarray(a, dtype=np.uint64)
    lo = a[..., 0].astype(object)
    hi = a[..., 1].astype(object)
    return lo + (hi << 64)


@dataclass
class Peel:
    sub: np.ndarray      # sub-round index of removal, per vertex
    alpha: int           # degeneracy
    subrounds: int


def peel(g) -> Peel:
    lib = _load()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    sub = np.zeros(max(g.n, 1), dtype=np.int32)
    alpha = np.zeros(1, dtype=np.int32)
    r = lib.orc_peel(g.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(sub, C.c_int32),
                     _p(alpha, C.c_int32))
    return Peel(sub[: g.n].copy(), int(alpha[0]), int(r))


def out_degrees(g, key: np.ndarray) -> np.ndarray:
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    fwd = (key[src] < key[dst]) | ((key[src] == key[dst]) & (src < dst))
    return np.bincount(src[fwd], minlength=g.n)


@dataclass
class Result:
    glob: list                       # C_0..C_{kcap-1} as Python ints
    glob_ovf: np.ndarray
    vertex: np.ndarray | None = None     # [n][K][2] uint64 limbs
    vertex_ovf: np.ndarray | None = None
    edge: np.ndarray | None = None       # [m][K][2] uint64 limbs
    edge_ovf: np.ndarray | None = None
    hist: np.ndarray | None = None
    stats: dict = field(default_factory=dict)

    @property
    def omega(self) -> int:
        return int(self.stats["omega"])


def count(g, key=None, prio=None, roots=None, kmax: int = 0, vertex=None, edge=None,
          hist_dim: int = 0) -> Result:
    """Run the oracle.  vertex / edge: None or (k_lo, k_hi)."""
    lib = _load()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    subrounds = 0
    if key is None:
        pe = peel(g)
        key = pe.sub
        subrounds = pe.subrounds
    key = np.ascontiguousarray(key, dtype=np.int32)
    alpha = int(out_degrees(g, key).max()) if g.n else 0
    kcap = alpha + 3
    prio_a = None if prio is None else np.ascontiguousarray(prio, dtype=np.int32)
    roots_a = None if roots is None else np.ascontiguousarray(roots, dtype=np.int32)
    glob = np.zeros((kcap, 2), dtype=np.uint64)
    govf = np.zeros(kcap, dtype=np.uint8)
    vc = vovf = ec = eovf = None
    vlo = vhi = elo = ehi = 0
    if vertex is not None:
        vlo, vhi = vertex
        vc = np.zeros((g.n, vhi - vlo + 1, 2), dtype=np.uint64)
        vovf = np.zeros(vhi - vlo + 1, dtype=np.uint8)
    if edge is not None:
        elo, ehi = edge
        ec = np.zeros((g.m, ehi - elo + 1, 2), dtype=np.uint64)
        eovf = np.zeros(ehi - elo + 1, dtype=np.uint8)
    hist = np.zeros((hist_dim, hist_dim), dtype=np.uint64) if hist_dim else None
    stats = np.zeros(12, dtype=np.uint64)
    rc = lib.orc_count(g.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(key, C.c_int32),
                       _p(prio_a, C.c_int32), _p(roots_a, C.c_int32),
                       0 if roots_a is None else int(roots_a.shape[0]), int(kmax),
                       kcap, _p(glob, C.c_uint64), _p(govf, C.c_uint8),
                       vlo, vhi, _p(vc, C.c_uint64), _p(vovf, C.c_uint8),
                       elo, ehi, _p(ec, C.c_uint64), _p(eovf, C.c_uint8),
                       hist_dim, _p(hist, C.c_uint64), _p(stats, C.c_uint64))
    if rc != 0:
        raise RuntimeError(f"oracle failed with status {rc}")
    names = ["nodes", "leaves", "alpha", "omega", "max_depth", "work_sw", "subrounds",
             "need_kcap", "hist_out", "work_child", "leaf_hp", "leaf_pairs"]
    st = {k: int(v) for k, v in zip(names, stats)}
    if key is not None and subrounds:
        st["subrounds"] = subrounds
    return Result(list(limbs_to_int(glob)), govf, vc, vovf, ec, eovf, hist, st)


def counts_exact(g, key=None, roots=None, kmax: int = 0) -> tuple[list[int], int]:
    """Global counts of any width: the oracle's own walk records the SCT leaf
    histogram L[h][p] (the leaves of Alg. 1; with kmax, the truncated tree
    of Sec. 5), and Sec. 5's read-off C_k = sum over h, p of L[h][p] C(p, k - h)
    is evaluated with exact Python integers.  C_0 = 1 for the whole graph
    (the empty clique), 0 for a root subset.  Returns (C_0..C_omega, omega)."""
    import math
    key_a = peel(g).sub if key is None else key
    alpha = int(out_degrees(g, key_a).max()) if g.n else 0
    hd = alpha + 2
    r = count(g, key=key_a, roots=roots, kmax=kmax, hist_dim=hd)
    if r.stats["hist_out"]:
        raise RuntimeError("leaf outside the histogram")
    L = r.hist
    omega = r.omega
    top = min(omega, kmax) if kmax else omega
    out = [0] * (top + 1)
    out[0] = 0 if roots is not None else 1
    nz = [(h, p, int(L[h, p])) for h, p in zip(*np.nonzero(L))]
    for k in range(1, top + 1):
        out[k] = sum(c * math.comb(p, k - h) for h, p, c in nz if 0 <= k - h <= p)
    return out, (top if kmax else omega)


def frequency(limbs: np.ndarray) -> list[tuple[int, int]]:
    """f(b) of one column of local counts (Sec. 6, demonstrations): the
    distinct values b in increasing order with the number of rows holding
    each.  limbs: [rows][2] uint64 (lo, hi) as count() returns them."""
    from collections import Counter
    vals = [int(lo) | (int(hi) << 64) for lo, hi in np.asarray(limbs, dtype=np.uint64).reshape(-1, 2)]
    return sorted(Counter(vals).items())

