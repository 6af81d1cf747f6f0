"""The allocation-free entry point pv_local_frequency_static, through the C
ABI: its output equals pv_local_frequency's on two calls in a row, the
second with a smaller input (the fixed scratch keeps the first call's
contents), and sizes beyond its scratch are refused."""
import sys

import numpy as np
import pytest

from paper_2001_06784_amd import graphgen as gg
from paper_2001_06784_amd import pivoter as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _table(ctx, g, klo, khi):
    import torch
    h = P.pv_graph_load_csr(ctx, g.n, g.row_ptr, g.col)
    dev = torch.zeros((g.n, khi - klo + 1, 2), dtype=torch.int64, device="cuda:0")
    try:
        res, lov = P.pv_count(h, local_kind=P.PV_VERTEX, k_lo=klo, k_hi=khi, local_out=dev.data_ptr())
        torch.cuda.synchronize()
    finally:
        P.pv_graph_free(h)
    assert lov == 0
    return dev


def test_static_frequency_equals_allocating_one():
    import torch
    ctx = P.pv_init(0)
    try:
        big = gg.plant_cliques(gg.chung_lu(60_000, 14, 2.3, 2000, 301), [45, 30], 302)
        small = gg.plant_cliques(gg.gnp(700, 0.03, 303), [14], 304)
        for g in (big, small):  # the second call is smaller than the first
            dev = _table(ctx, g, 3, 8)
            for col in range(6):
                want_v, want_f = P.pv_local_frequency(ctx, dev.data_ptr(), g.n, 6, col)
                got_v, got_f = P.pv_local_frequency_static(ctx, dev.data_ptr(), g.n, 6, col)
                assert got_v == want_v and np.array_equal(got_f, want_f), (g.n, col)
                assert int(got_f.sum()) == g.n
            _say(f"[no-alloc] n={g.n}: {len(got_v)} distinct values of the k=8 counts")
        # the largest size the scratch holds, and one more row
        rows = P.PV_FREQ_STATIC_ROWS
        dev = torch.zeros((rows + 1, 1, 2), dtype=torch.int64, device="cuda:0")
        dev[:, 0, 0] = torch.arange(rows + 1, device="cuda:0") % 7
        got_v, got_f = P.pv_local_frequency_static(ctx, dev.data_ptr(), rows, 1, 0)
        assert got_v == list(range(7)) and int(got_f.sum()) == rows
        with pytest.raises(P.PivoterError) as ei:
            P.pv_local_frequency_static(ctx, dev.data_ptr(), rows + 1, 1, 0)
        assert ei.value.status == P.PV_ETOOBIG
        # a buffer too small: the count is reported, nothing else written
        with pytest.raises(P.PivoterError) as ei:
            P.pv_local_frequency_static(ctx, dev.data_ptr(), rows, 1, 0, cap=3)
        assert ei.value.status == P.PV_EBUFSIZE
    finally:
        P.pv_fini(ctx)
