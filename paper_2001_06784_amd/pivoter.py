"""Thin ctypes binding of libpivoter (include/pivoter.h), same names as the
C ABI.  Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  Importing this module does not touch the GPU; the
first call loads libpivoter.so and raises if it is missing (there is no
fallback path).

Device buffers are passed as integer device addresses (for example
``tensor.data_ptr()`` of a torch tensor on the same device); host buffers as
numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpivoter.so")

PV_OK = 0
PV_EINVAL = -1
PV_ENOTSIMPLE = -2
PV_ENOMEM = -3
PV_EOVERFLOW = -4
PV_EDEVICE = -5
PV_ETOOBIG = -6
PV_EBUFSIZE = -7
PV_ECANCELLED = -8
PV_EAGAIN = -9
PV_ETIMEDOUT = -10

PV_NONE, PV_VERTEX, PV_EDGE = 0, 1, 2
PV_TRUST_INPUT = 1
PV_DEDUP = 2
PV_SYMMETRIZE = 4
PV_MAX_ALPHA = 4096
PV_MAX_LOCAL_K = 16
PV_FREQ_STATIC_ROWS = 1 << 20

# every function declared in include/pivoter.h
ABI_FUNCTIONS = [
    "pv_strerror", "pv_init", "pv_fini", "pv_cancel", "pv_memory", "pv_measure_peaks", "pv_set_stream", "pv_set_dfs_max", "pv_set_dfs_budget", "pv_set_lane_max",
    "pv_set_timing",
    "pv_last_error",
    "pv_graph_load_csr", "pv_graph_load_csr_device", "pv_graph_free", "pv_graph_size",
    "pv_graph_orient", "pv_graph_export_order", "pv_count_global", "pv_count_global_wide", "pv_count_local",
    "pv_local_frequency", "pv_local_frequency_static",
    "pv_graph_edge_list", "pv_count", "pv_count_roots", "pv_count_batch", "pv_count_global_batch",
    "pv_server_start", "pv_server_submit", "pv_server_wait", "pv_server_poll", "pv_server_cancel",
    "pv_server_stats", "pv_server_stop", "pv_autotune", "pv_tune_key",
]

PV_REQ_GLOBAL, PV_REQ_VERTEX = 0, 1


class pv_u128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_uint64)]


class pv_stats(C.Structure):
    _fields_ = [("nodes", C.c_uint64), ("leaves", C.c_uint64), ("items", C.c_uint64),
                ("work", C.c_uint64), ("alpha", C.c_int32), ("omega", C.c_int32),
                ("subrounds", C.c_int32), ("truncated", C.c_int32), ("levels", C.c_int32),
                ("ms_peel", C.c_float), ("ms_orient", C.c_float), ("ms_levels", C.c_float),
                ("ms_finalize", C.c_float), ("launches_kind", C.c_uint32 * 3),
                ("ms_kind", C.c_float * 3), ("work_kind", C.c_uint64 * 3),
                ("kernel_kl", C.c_int32), ("kernel_lk", C.c_int32), ("attempts", C.c_int32),
                ("child_work", C.c_uint64), ("leaf_hp", C.c_uint64), ("leaf_pp", C.c_uint64),
                ("heavy_chunks", C.c_int32)]

    def as_dict(self) -> dict:
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v) if isinstance(v, C.Array) else v
        return d


class pv_peaks(C.Structure):
    _fields_ = [("hbm_copy_gbs", C.c_double), ("hbm_read_gbs", C.c_double), ("lds_read_gbs", C.c_double),
                ("valu_gops", C.c_double), ("ms_copy", C.c_float), ("ms_read", C.c_float),
                ("ms_lds", C.c_float), ("ms_valu", C.c_float)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class pv_config(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("hbm_budget", C.c_int64), ("tune_cache", C.c_char_p),
                ("dfs_max", C.c_int32), ("dfs_budget", C.c_int32), ("lane_max", C.c_int32),
                ("timeout_ms", C.c_int32)]


class pv_tune(C.Structure):
    _fields_ = [("dfs_max", C.c_int32), ("dfs_budget", C.c_int32), ("lane_max", C.c_int32),
                ("ms_best", C.c_float), ("ms_default", C.c_float), ("trials", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class pv_server_cfg(C.Structure):
    _fields_ = [("device", C.c_int32), ("workers", C.c_int32), ("max_batch", C.c_int32),
                ("cache_bytes", C.c_int64), ("batch_bytes", C.c_int64)]


class pv_request(C.Structure):
    _fields_ = [("graph_key", C.c_uint64), ("n", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("kind", C.c_int32), ("k_lo", C.c_int32), ("k_hi", C.c_int32),
                ("counts", C.POINTER(pv_u128)), ("cap", C.c_int32),
                ("vertex_out", C.POINTER(pv_u128))]


class pv_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("omega", C.c_int32), ("overflow", C.c_uint64),
                ("local_overflow", C.c_uint64), ("queue_us", C.c_double), ("run_us", C.c_double),
                ("total_us", C.c_double), ("batch_size", C.c_int32)]


class PivoterError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = ""
        try:
            detail = _lib().pv_last_error().decode()
        except Exception:  # noqa: BLE001 - diagnostics only
            pass
        super().__init__(f"{what}: {_lib().pv_strerror(status).decode()} ({status})"
                         + (f" [{detail}]" if detail else ""))


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2001_06784_amd.build")
        # PyTorch-ROCm ships its own libamdhip64.so.7.  Loading it first makes
        # libpivoter bind to that same runtime (identical SONAME), so torch
        # tensors and library calls share one HIP runtime in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
        pvp = C.POINTER(C.c_void_p)
        u128p = C.POINTER(pv_u128)
        u64p = C.POINTER(C.c_uint64)
        i32p = C.POINTER(C.c_int32)
        sp = C.POINTER(pv_stats)
        sig = {
            "pv_strerror": (C.c_char_p, [i32]),
            "pv_last_error": (C.c_char_p, []),
            "pv_init": (i32, [i32, C.POINTER(pv_config), pvp]),
            "pv_fini": (None, [vp]),
            "pv_cancel": (i32, [vp]),
            "pv_memory": (i32, [vp, C.POINTER(C.c_int64)]),
            "pv_measure_peaks": (i32, [vp, C.c_int64, C.POINTER(pv_peaks)]),
            "pv_set_stream": (i32, [vp, vp]),
            "pv_set_dfs_max": (i32, [vp, i32]),
            "pv_set_timing": (i32, [vp, i32]),
            "pv_set_dfs_budget": (i32, [vp, i32]),
            "pv_set_lane_max": (i32, [vp, i32]),
            "pv_graph_load_csr": (i32, [vp, i32, i32p, i32p, u32, pvp]),
            "pv_graph_load_csr_device": (i32, [vp, i32, i64, vp, vp, u32, pvp]),
            "pv_graph_free": (i32, [vp]),
            "pv_graph_size": (i32, [vp, i32p, C.POINTER(C.c_int64)]),
            "pv_graph_orient": (i32, [vp, i32p]),
            "pv_graph_export_order": (i32, [vp, i32p]),
            "pv_count_global": (i32, [vp, i32, u128p, i32, i32p, u64p, sp]),
            "pv_count_global_wide": (i32, [vp, i32, u64p, i32, i32, i32p, u64p, sp]),
            "pv_local_frequency": (i32, [vp, vp, i64, i32, i32, u128p, u64p, i64, C.POINTER(C.c_int64)]),
            "pv_local_frequency_static": (i32, [vp, vp, i64, i32, i32, u128p, u64p, i64, C.POINTER(C.c_int64)]),
            "pv_count_local": (i32, [vp, i32, i32, i32, u128p, i64, u64p, sp]),
            "pv_graph_edge_list": (i32, [vp, i32p, i32p]),
            "pv_count": (i32, [vp, i32, i32, u128p, i32, i32p, u64p, i32, i32, i32, vp, u64p, sp]),
            "pv_count_roots": (i32, [vp, i32p, i32, i32, u128p, i32, i32p, u64p, i32, i32, i32, vp, u64p, sp]),
            "pv_count_batch": (i32, [vp, i32, pvp, i32, u128p, i32, i32p, u64p, i32, i32, i32, vp,
                                     u64p, i32p, sp]),
            "pv_count_global_batch": (i32, [vp, i32, pvp, i32, u128p, i32, i32p, u64p, i32p, sp]),
            "pv_autotune": (i32, [vp, i32, i32, i32, vp, i32, C.POINTER(pv_tune)]),
            "pv_tune_key": (C.c_char_p, [vp, i32, i32, i32]),
            "pv_server_start": (i32, [C.POINTER(pv_server_cfg), pvp]),
            "pv_server_submit": (i32, [vp, C.POINTER(pv_request), u64p]),
            "pv_server_wait": (i32, [vp, C.c_uint64, i64, C.POINTER(pv_result)]),
            "pv_server_poll": (i32, [vp, C.c_uint64, C.POINTER(pv_result)]),
            "pv_server_cancel": (i32, [vp, C.c_uint64]),
            "pv_server_stats": (i32, [vp, i32p, C.POINTER(C.c_int64), i32p]),
            "pv_server_stop": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def load_library():
    """Load libpivoter.so now (raises ImportError if it is not built)."""
    return _lib()


def _check(status: int, what: str, allow=()):
    if status != PV_OK and status not in allow:
        raise PivoterError(status, what)
    return status


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def u128_to_ints(arr) -> list:
    """ctypes pv_u128 array or (..., 2) uint64 array -> Python ints."""
    a = np.asarray(arr)
    if a.dtype.fields is not None:
        a = np.frombuffer(a.tobytes(), dtype=np.uint64).reshape(-1, 2)
    lo = a[..., 0].astype(object)
    hi = a[..., 1].astype(object)
    return (lo + (hi << 64)).tolist()


# ------------------------------------------------------------- functions

def pv_strerror(status: int) -> str:
    return _lib().pv_strerror(status).decode()


def pv_last_error() -> str:
    return _lib().pv_last_error().decode()


def pv_init(device: int = 0, stream: int | None = None, hbm_budget: int = 0, tune_cache: str | None = None,
            dfs_max: int = 0, dfs_budget: int = 0, lane_max: int = 0, timeout_ms: int = 0) -> int:
    cfg = pv_config(stream, hbm_budget, tune_cache.encode() if tune_cache else None, dfs_max, dfs_budget,
                    lane_max, timeout_ms)
    out = C.c_void_p()
    _check(_lib().pv_init(device, C.byref(cfg), C.byref(out)), "pv_init")
    return out.value


def pv_fini(ctx: int) -> None:
    _lib().pv_fini(ctx)


def pv_cancel(ctx: int) -> None:
    """Cancel the count call running on ctx now (from any thread)."""
    _check(_lib().pv_cancel(ctx), "pv_cancel")


def pv_memory(ctx: int) -> int:
    b = C.c_int64()
    _check(_lib().pv_memory(ctx, C.byref(b)), "pv_memory")
    return b.value


def pv_measure_peaks(ctx: int, copy_bytes: int = 0) -> dict:
    """The device's measured HBM copy/read, LDS read and VALU rates."""
    out = pv_peaks()
    _check(_lib().pv_measure_peaks(ctx, copy_bytes, C.byref(out)), "pv_measure_peaks")
    return out.as_dict()


def pv_set_stream(ctx: int, stream: int | None) -> None:
    _check(_lib().pv_set_stream(ctx, stream), "pv_set_stream")


def pv_set_dfs_max(ctx: int, dfs_max: int) -> None:
    _check(_lib().pv_set_dfs_max(ctx, dfs_max), "pv_set_dfs_max")


def pv_set_dfs_budget(ctx: int, nodes: int) -> None:
    _check(_lib().pv_set_dfs_budget(ctx, nodes), "pv_set_dfs_budget")


def pv_set_lane_max(ctx: int, lane_max: int) -> None:
    _check(_lib().pv_set_lane_max(ctx, lane_max), "pv_set_lane_max")


def pv_set_timing(ctx: int, on: bool) -> None:
    _check(_lib().pv_set_timing(ctx, int(bool(on))), "pv_set_timing")


def pv_graph_load_csr(ctx: int, n: int, row_ptr, col, flags: int = 0) -> int:
    rp, rpp = _i32(row_ptr)
    cl, clp = _i32(col if len(col) else np.zeros(1, np.int32))
    if rp.shape[0] != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    out = C.c_void_p()
    _check(_lib().pv_graph_load_csr(ctx, n, rpp, clp, flags, C.byref(out)), "pv_graph_load_csr")
    return out.value


def pv_graph_load_csr_device(ctx: int, n: int, nnz: int, d_row_ptr: int, d_col: int,
                             flags: int = 0) -> int:
    out = C.c_void_p()
    _check(_lib().pv_graph_load_csr_device(ctx, n, nnz, d_row_ptr, d_col, flags, C.byref(out)),
           "pv_graph_load_csr_device")
    return out.value


def pv_graph_free(g: int) -> int:
    """Returns PV_OK, or PV_EAGAIN while a count on another thread uses g."""
    return _check(_lib().pv_graph_free(g), "pv_graph_free", allow=(PV_EAGAIN,))


def pv_graph_size(g: int) -> tuple[int, int]:
    n = C.c_int32()
    m = C.c_int64()
    _check(_lib().pv_graph_size(g, C.byref(n), C.byref(m)), "pv_graph_size")
    return n.value, m.value


def pv_graph_orient(g: int) -> int:
    a = C.c_int32()
    _check(_lib().pv_graph_orient(g, C.byref(a)), "pv_graph_orient")
    return a.value


def pv_graph_export_order(g: int) -> np.ndarray:
    n, _ = pv_graph_size(g)
    out = np.zeros(max(n, 1), dtype=np.int32)
    _check(_lib().pv_graph_export_order(g, out.ctypes.data_as(C.POINTER(C.c_int32))),
           "pv_graph_export_order")
    return out[:n]


@dataclass
class GlobalResult:
    counts: list          # C_0..C_{cap-1} as Python ints
    omega: int
    overflow: list        # k with C_k >= 2^128
    stats: dict
    status: int


def pv_count_global(g: int, k_max: int = 0, cap: int = PV_MAX_ALPHA + 2) -> GlobalResult:
    counts = (pv_u128 * cap)()
    ov = (C.c_uint64 * ((cap + 63) // 64))()
    om = C.c_int32()
    st = pv_stats()
    s = _check(_lib().pv_count_global(g, k_max, counts, cap, C.byref(om), ov, C.byref(st)),
               "pv_count_global", allow=(PV_EOVERFLOW,))
    ovf = [k for k in range(cap) if (ov[k >> 6] >> (k & 63)) & 1]
    return GlobalResult(u128_to_ints(counts), om.value, ovf, st.as_dict(), s)


def pv_count_global_wide(g: int, k_max: int = 0, cap: int = PV_MAX_ALPHA + 2, limbs: int = 4) -> GlobalResult:
    """Global counts in `limbs` 64-bit limbs per k, as Python ints."""
    counts = np.zeros((max(cap, 1), limbs), dtype=np.uint64)
    ov = (C.c_uint64 * ((cap + 63) // 64))()
    om = C.c_int32()
    st = pv_stats()
    s = _check(_lib().pv_count_global_wide(g, k_max, counts.ctypes.data_as(C.POINTER(C.c_uint64)), cap, limbs,
                                           C.byref(om), ov, C.byref(st)),
               "pv_count_global_wide", allow=(PV_EOVERFLOW,))
    ovf = [k for k in range(cap) if (ov[k >> 6] >> (k & 63)) & 1]
    vals = [sum(int(counts[k, i]) << (64 * i) for i in range(limbs)) for k in range(cap)]
    return GlobalResult(vals, om.value, ovf, st.as_dict(), s)


def pv_local_frequency(ctx: int, local_ptr: int, rows: int, K: int, col: int):
    """Distinct values of column `col` of a device [rows][K] u128 table, in
    increasing order (Python ints), and how many rows hold each (uint64)."""
    cap = max(rows, 1)
    vals = np.zeros((cap, 2), dtype=np.uint64)
    freq = np.zeros(cap, dtype=np.uint64)
    nd = C.c_int64()
    _check(_lib().pv_local_frequency(ctx, local_ptr, rows, K, col, vals.ctypes.data_as(C.POINTER(pv_u128)),
                                     freq.ctypes.data_as(C.POINTER(C.c_uint64)), cap, C.byref(nd)),
           "pv_local_frequency")
    D = nd.value
    return [int(vals[i, 0]) | (int(vals[i, 1]) << 64) for i in range(D)], freq[:D]


def pv_local_frequency_static(ctx: int, local_ptr: int, rows: int, K: int, col: int, cap: int | None = None):
    """pv_local_frequency on the library's fixed scratch (no allocation)."""
    cap = max(rows, 1) if cap is None else cap
    vals = np.zeros((max(cap, 1), 2), dtype=np.uint64)
    freq = np.zeros(max(cap, 1), dtype=np.uint64)
    nd = C.c_int64()
    _check(_lib().pv_local_frequency_static(ctx, local_ptr, rows, K, col, vals.ctypes.data_as(C.POINTER(pv_u128)),
                                            freq.ctypes.data_as(C.POINTER(C.c_uint64)), cap, C.byref(nd)),
           "pv_local_frequency_static")
    D = nd.value
    return [int(vals[i, 0]) | (int(vals[i, 1]) << 64) for i in range(D)], freq[:D]


def pv_count_local(g: int, kind: int, k_lo: int, k_hi: int):
    """Returns ((rows, K, 2) uint64 limbs, overflow word, stats)."""
    n, m = pv_graph_size(g)
    K = k_hi - k_lo + 1
    rows = n if kind == PV_VERTEX else m
    out = np.zeros((max(rows, 1), K, 2), dtype=np.uint64)
    ov = C.c_uint64()
    st = pv_stats()
    _check(_lib().pv_count_local(g, kind, k_lo, k_hi, out.ctypes.data_as(C.POINTER(pv_u128)),
                                 rows * K, C.byref(ov), C.byref(st)),
           "pv_count_local", allow=(PV_EOVERFLOW,))
    return out[:rows], ov.value, st.as_dict()


def pv_graph_edge_list(g: int) -> tuple[np.ndarray, np.ndarray]:
    _, m = pv_graph_size(g)
    u = np.zeros(max(m, 1), dtype=np.int32)
    v = np.zeros(max(m, 1), dtype=np.int32)
    _check(_lib().pv_graph_edge_list(g, u.ctypes.data_as(C.POINTER(C.c_int32)),
                                     v.ctypes.data_as(C.POINTER(C.c_int32))), "pv_graph_edge_list")
    return u[:m], v[:m]


def pv_count(g: int, reorient: bool = False, k_max: int = 0, cap: int = PV_MAX_ALPHA + 2,
             local_kind: int = PV_NONE, k_lo: int = 0, k_hi: int = 0, local_out: int | None = None):
    """One pass: global counts (host) and optional local counts into the
    device buffer `local_out` (address).  Returns (GlobalResult, local overflow word)."""
    counts = (pv_u128 * cap)()
    ov = (C.c_uint64 * ((cap + 63) // 64))()
    om = C.c_int32()
    lov = C.c_uint64()
    st = pv_stats()
    s = _check(_lib().pv_count(g, int(reorient), k_max, counts, cap, C.byref(om), ov, local_kind,
                               k_lo, k_hi, local_out, C.byref(lov), C.byref(st)),
               "pv_count", allow=(PV_EOVERFLOW,))
    ovf = [k for k in range(cap) if (ov[k >> 6] >> (k & 63)) & 1]
    return GlobalResult(u128_to_ints(counts), om.value, ovf, st.as_dict(), s), lov.value


def pv_count_roots(g: int, roots, k_max: int = 0, cap: int = PV_MAX_ALPHA + 2, local_kind: int = PV_NONE,
                   k_lo: int = 0, k_hi: int = 0, local_out: int | None = None, with_local_ovf: bool = False):
    """Counts of the cliques whose smallest-key vertex is one of `roots`;
    local counts go to the device buffer `local_out` (address).  Returns a
    GlobalResult, or (GlobalResult, local overflow word) with_local_ovf."""
    r, rp = _i32(roots if len(roots) else np.zeros(1, np.int32))
    counts = (pv_u128 * cap)()
    ov = (C.c_uint64 * ((cap + 63) // 64))()
    om = C.c_int32()
    lov = C.c_uint64()
    st = pv_stats()
    s = _check(_lib().pv_count_roots(g, rp, len(roots), k_max, counts, cap, C.byref(om), ov, local_kind,
                                     k_lo, k_hi, local_out, C.byref(lov), C.byref(st)),
               "pv_count_roots", allow=(PV_EOVERFLOW,))
    ovf = [k for k in range(cap) if (ov[k >> 6] >> (k & 63)) & 1]
    res = GlobalResult(u128_to_ints(counts), om.value, ovf, st.as_dict(), s)
    return (res, lov.value) if with_local_ovf else res


def pv_count_global_batch_raw(ctx: int, graphs, k_max: int = 0, cap: int = 256):
    """Batched global counts, results as arrays: counts (G, cap, 2) uint64
    limbs, omega (G,) int32, overflow words (G, (cap+63)//64) uint64, status,
    stats."""
    G = len(graphs)
    arr = (C.c_void_p * max(G, 1))(*graphs)
    nw = (cap + 63) // 64
    counts = np.zeros((max(G, 1), cap, 2), dtype=np.uint64)
    om = np.zeros(max(G, 1), dtype=np.int32)
    ov = np.zeros((max(G, 1), nw), dtype=np.uint64)
    gst = np.zeros(max(G, 1), dtype=np.int32)
    st = pv_stats()
    s = _check(_lib().pv_count_global_batch(ctx, G, arr, k_max,
                                            counts.ctypes.data_as(C.POINTER(pv_u128)), cap,
                                            om.ctypes.data_as(C.POINTER(C.c_int32)),
                                            ov.ctypes.data_as(C.POINTER(C.c_uint64)),
                                            gst.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(st)),
               "pv_count_global_batch", allow=(PV_EOVERFLOW, PV_EBUFSIZE))
    d = st.as_dict()
    d["status"] = gst[:G].tolist()
    return counts[:G], om[:G], ov[:G], s, d


def pv_count_global_batch(ctx: int, graphs, k_max: int = 0, cap: int = 256):
    """Batched global counts: ([GlobalResult per graph], stats)."""
    counts, om, ov, s, st = pv_count_global_batch_raw(ctx, graphs, k_max, cap)
    out = []
    for i in range(len(graphs)):
        ovf = [k for k in range(cap) if (int(ov[i, k >> 6]) >> (k & 63)) & 1]
        out.append(GlobalResult(u128_to_ints(counts[i]), int(om[i]), ovf, {}, s))
    return out, st


def pv_count_batch(ctx: int, graphs, k_max: int = 0, cap: int = 256, local_kind: int = PV_NONE,
                   k_lo: int = 0, k_hi: int = 0, local_out: int | None = None):
    """Batched counts with optional per-vertex counts into the device buffer
    `local_out` ((sum of n) x K u128).  Returns (counts (G, cap, 2) uint64,
    omega, overflow words, status, local overflow word, stats)."""
    G = len(graphs)
    arr = (C.c_void_p * max(G, 1))(*graphs)
    nw = (cap + 63) // 64
    counts = np.zeros((max(G, 1), cap, 2), dtype=np.uint64)
    om = np.zeros(max(G, 1), dtype=np.int32)
    ov = np.zeros((max(G, 1), nw), dtype=np.uint64)
    lov = C.c_uint64()
    gst = np.zeros(max(G, 1), dtype=np.int32)
    st = pv_stats()
    s = _check(_lib().pv_count_batch(ctx, G, arr, k_max, counts.ctypes.data_as(C.POINTER(pv_u128)),
                                     cap, om.ctypes.data_as(C.POINTER(C.c_int32)),
                                     ov.ctypes.data_as(C.POINTER(C.c_uint64)), local_kind, k_lo, k_hi,
                                     local_out, C.byref(lov), gst.ctypes.data_as(C.POINTER(C.c_int32)),
                                     C.byref(st)),
               "pv_count_batch", allow=(PV_EOVERFLOW, PV_EBUFSIZE))
    d = st.as_dict()
    d["status"] = gst[:G].tolist()
    return counts[:G], om[:G], ov[:G], s, lov.value, d


def pv_autotune(g: int, local_kind: int = PV_NONE, k_lo: int = 0, k_hi: int = 0,
                local_out: int | None = None, reps: int = 2) -> dict:
    t = pv_tune()
    _check(_lib().pv_autotune(g, local_kind, k_lo, k_hi, local_out, reps, C.byref(t)), "pv_autotune")
    return t.as_dict()


def pv_tune_key(g: int, local_kind: int = PV_NONE, k_lo: int = 0, k_hi: int = 0) -> str:
    return _lib().pv_tune_key(g, local_kind, k_lo, k_hi).decode()


class Server:
    """The library's request loop (pv_server_*).  Requests keep references to
    their CSR and output arrays until they complete."""

    def __init__(self, device: int = 0, workers: int = 2, max_batch: int = 64,
                 cache_bytes: int = 8 << 30, batch_bytes: int = 4 << 30):
        cfg = pv_server_cfg(device, workers, max_batch, cache_bytes, batch_bytes)
        h = C.c_void_p()
        _check(_lib().pv_server_start(C.byref(cfg), C.byref(h)), "pv_server_start")
        self.h = h
        self._live = {}

    def submit(self, key: int, g, kind: int = PV_REQ_GLOBAL, k_lo: int = 0, k_hi: int = 0,
               cap: int = PV_MAX_ALPHA + 2) -> int:
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(g.col if len(g.col) else np.zeros(1, np.int32), dtype=np.int32)
        counts = np.zeros((cap, 2), dtype=np.uint64)
        vout = None
        if kind == PV_REQ_VERTEX:
            vout = np.zeros((max(g.n, 1), k_hi - k_lo + 1, 2), dtype=np.uint64)
        req = pv_request(key, g.n, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                         col.ctypes.data_as(C.POINTER(C.c_int32)), kind, k_lo, k_hi,
                         counts.ctypes.data_as(C.POINTER(pv_u128)), cap,
                         vout.ctypes.data_as(C.POINTER(pv_u128)) if vout is not None else None)
        t = C.c_uint64()
        _check(_lib().pv_server_submit(self.h, C.byref(req), C.byref(t)), "pv_server_submit")
        self._live[t.value] = (rp, col, counts, vout, g.n)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        """(status, GlobalResult-like dict, vertex counts or None, result struct)."""
        r = pv_result()
        s = _lib().pv_server_wait(self.h, ticket, timeout_us, C.byref(r))
        if s == PV_EAGAIN:
            return None
        _check(s, "pv_server_wait")
        rp, col, counts, vout, n = self._live.pop(ticket)
        return r, counts, (vout[:n] if vout is not None else None)

    def cancel(self, ticket: int) -> int:
        return _lib().pv_server_cancel(self.h, ticket)

    def stats(self):
        res, by, pend = C.c_int32(), C.c_int64(), C.c_int32()
        _check(_lib().pv_server_stats(self.h, C.byref(res), C.byref(by), C.byref(pend)), "pv_server_stats")
        return res.value, by.value, pend.value

    def stop(self):
        if self.h:
            _lib().pv_server_stop(self.h)
            self.h = None
            self._live.clear()

