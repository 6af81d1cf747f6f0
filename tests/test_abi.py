"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs on machines without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2001_06784_amd import pivoter as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "pivoter.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(pv_\w+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    decl = _declared()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(lib, name), name
    # the binding covers exactly the declared ABI
    assert sorted(P.ABI_FUNCTIONS) == decl


def test_status_strings_are_static_and_distinct():
    msgs = {s: P.pv_strerror(s) for s in range(-9, 1)}
    assert len(set(msgs.values())) == len(msgs)
    assert P.pv_strerror(12345) == "unknown status"


def test_null_handles_are_rejected_without_touching_the_device():
    lib = P.load_library()
    assert lib.pv_graph_orient(None, None) == P.PV_EINVAL
    assert lib.pv_count_global(None, 0, None, 0, None, None, None) == P.PV_EINVAL
    assert lib.pv_set_stream(None, None) == P.PV_EINVAL
    assert lib.pv_set_dfs_max(None, 8) == P.PV_EINVAL
    assert lib.pv_graph_size(None, None, None) == P.PV_EINVAL
    assert lib.pv_graph_free(None) == P.PV_OK
    lib.pv_fini(None)
    assert lib.pv_memory(None, None) == P.PV_EINVAL
    assert lib.pv_autotune(None, 0, 0, 0, None, 1, None) == P.PV_EINVAL
    assert lib.pv_count_roots(None, None, 0, 0, None, 0, None, None, 0, 0, 0, None, None, None) == P.PV_EINVAL
    assert lib.pv_count_global_batch(None, 0, None, 0, None, 0, None, None, None, None) == P.PV_EINVAL
    assert lib.pv_tune_key(None, 0, 0, 0) == b""


def test_header_constants_match_binding():
    hdr = open(os.path.join(ROOT, "include", "pivoter.h")).read()
    for name in ["PV_OK", "PV_EINVAL", "PV_ENOTSIMPLE", "PV_ENOMEM", "PV_EOVERFLOW", "PV_EDEVICE",
                 "PV_ETOOBIG", "PV_EBUFSIZE", "PV_ECANCELLED", "PV_EAGAIN", "PV_ETIMEDOUT", "PV_NONE", "PV_VERTEX",
                 "PV_EDGE", "PV_MAX_ALPHA", "PV_MAX_LOCAL_K", "PV_TRUST_INPUT", "PV_DEDUP",
                 "PV_SYMMETRIZE"]:
        m = re.search(rf"#define {name}\s+(-?\d+)u?\b", hdr)
        assert m, name
        assert int(m.group(1)) == getattr(P, name), name
    assert "#define PV_FREQ_STATIC_ROWS (1 << 20)" in hdr and P.PV_FREQ_STATIC_ROWS == 1 << 20
    assert ctypes.sizeof(P.pv_u128) == 16
    assert ctypes.sizeof(P.pv_stats) == 168
    assert ctypes.sizeof(P.pv_config) == 40
    assert ctypes.sizeof(P.pv_tune) == 24
