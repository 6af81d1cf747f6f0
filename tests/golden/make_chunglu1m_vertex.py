"""Writes chunglu1m_vertex3-10.json: the oracle's whole-graph results on the
benchmark workload (Chung-Lu, n = 1,000,000, average degree 20, exponent 2.3,
degree cap 20,000, seed 1; global counts for all k and per-vertex counts for
k = 3..10).  Only the oracle runs here, in the paper's parallel form (Sec. 5:
the root subproblems are independent, counted with private counters and
summed); nothing of the GPU library is loaded.

The per-vertex table (1M x 8 exact u128 counts, 128 MB) is stored as SHA-256
digests of its little-endian (lo, hi) uint64 limbs, whole and per column,
plus every column of a seeded sample of rows in full, so the GPU test can
compare its own table element by element through the digests.

    python tests/golden/make_chunglu1m_vertex.py [workers]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

K_LO, K_HI = 3, 10


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def sample_rows(n: int, degrees: np.ndarray) -> np.ndarray:
    rng = np.random.default_rng(5)
    top = np.argsort(-degrees, kind="stable")[:32]
    return np.unique(np.concatenate([rng.choice(n, 224, replace=False), top])).astype(np.int64)


def main():
    from oracle import oracle as O
    from oracle import parallel as OP
    from paper_2001_06784_amd import graphgen as gg

    workers = int(sys.argv[1]) if len(sys.argv) > 1 else None
    g = gg.chung_lu_social(n=1_000_000, avg_deg=20.0, gamma=2.3, max_deg=20_000.0, seed=1)
    t0 = time.perf_counter()
    pe = O.peel(g)
    t1 = time.perf_counter()
    r = OP.count_parallel(g, pe.sub, workers=workers, vertex=(K_LO, K_HI))
    t2 = time.perf_counter()
    vert = r["vertex"]
    st = r["stats"]
    assert r["overflow"] == 0
    rows = sample_rows(g.n, g.degrees())
    out = {
        "workload": "chung-lu n=1000000 avg_deg=20 gamma=2.3 max_deg=20000 seed=1; "
                    "global counts all k + per-vertex k=3..10",
        "writer": "tests/golden/make_chunglu1m_vertex.py (oracle only)",
        "n": int(g.n), "m": int(g.m), "alpha": int(pe.alpha), "subrounds": int(pe.subrounds),
        "omega": int(st["omega"]), "nodes": int(st["nodes"]), "leaves": int(st["leaves"]),
        "work_sw": int(st["work_sw"]),
        "glob": [str(int(x)) for x in r["glob"][: int(st["omega"]) + 1]],
        "k_lo": K_LO, "k_hi": K_HI,
        "vertex_sha256": digest(vert),
        "vertex_col_sha256": [digest(vert[:, c, :]) for c in range(K_HI - K_LO + 1)],
        "rows": {str(int(v)): [[str(int(vert[v, c, 0])), str(int(vert[v, c, 1]))]
                                for c in range(K_HI - K_LO + 1)] for v in rows},
        "oracle_seconds": {"peel": round(t1 - t0, 2), "count_wall": round(t2 - t1, 2),
                           "count_busy_summed": round(r["busy_s"], 2), "workers": r["workers"]},
    }
    with open(os.path.join(HERE, "chunglu1m_vertex3-10.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("n", "m", "alpha", "omega", "nodes", "leaves", "oracle_seconds")}))


if __name__ == "__main__":
    main()
