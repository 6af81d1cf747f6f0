"""Host-side checks that need no GPU: the benchmark's command line and the
seeded generators that feed both the oracle and the GPU path."""
import os
import subprocess
import sys

import numpy as np

from paper_2001_06784_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    # one GPU only: the request is refused before anything touches a device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_serving_workload_is_switched_off():
    # the serving benchmark refuses to run before it builds its pool or
    # loads the library
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "serve"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "disabled" in r.stderr


def test_rmat_web_plants_disjoint_cliques():
    # R-MAT plus planted cliques: every planted set is a clique, the sets are
    # disjoint, and the generator is deterministic for its seeds
    g = gg.rmat_web(scale=10, cliques=4, clique_lo=20, clique_hi=24)
    h = gg.rmat_web(scale=10, cliques=4, clique_lo=20, clique_hi=24)
    assert np.array_equal(g.row_ptr, h.row_ptr) and np.array_equal(g.col, h.col)
    sizes = gg._rng(2).integers(20, 25, 4)
    verts = gg._rng(3).permutation(g.n)[: int(sizes.sum())]
    off = 0
    seen = set()
    for s in sizes:
        vs = [int(v) for v in verts[off: off + s]]
        off += s
        assert not seen.intersection(vs)
        seen.update(vs)
        for a in vs:
            row = set(g.col[g.row_ptr[a]: g.row_ptr[a + 1]].tolist())
            assert all(b in row for b in vs if b != a)


def test_rmat_root_sample_matches_the_parity_sample():
    # the benchmark's stratified root sample: with scale 1 it is the sample
    # the sampled-root parity tests draw (same strata, seed and order), and a
    # larger scale keeps to the strata
    sys.path.insert(0, ROOT)
    import bench
    from oracle import oracle as O
    g = gg.rmat_web(scale=12, cliques=4, clique_lo=20, clique_hi=24)
    key = O.peel(g).sub
    roots, od = bench.rmat_root_sample(g, key, 1)
    assert np.array_equal(od, O.out_degrees(g, key))
    rng = np.random.default_rng(2022)
    want = []
    for lo, hi, cnt in [(0, 64, 2000), (64, 128, 40), (128, 256, 10), (256, 512, 5)]:
        pool = np.nonzero((od > lo) & (od <= hi))[0]
        want.append(rng.choice(pool, min(cnt, len(pool)), replace=False))
    want.append(np.nonzero(od == 0)[0][:5])
    assert np.array_equal(roots, np.concatenate(want).astype(np.int32))
    big, _ = bench.rmat_root_sample(g, key, 3)
    assert len(np.unique(big)) == len(big)
    assert len(big) >= len(roots) and od[big].max() <= 512
