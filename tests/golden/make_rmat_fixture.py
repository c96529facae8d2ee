"""Write the stored expected values of a large RMAT configuration.

The values come from the CPU oracle alone (``oracle/``) on the seeded input
of ``graphgen`` and are written to ``tests/golden/rmat<scale>_seed<seed>.json``;
GPU tests compare the library with them where running the oracle inside the
test would take too long (RMAT scale 26: about 20 minutes of oracle time).

Stored: sizes, T (Eq. 2), the work counts, SHA-256 digests of the oracle's
upper-triangular CSR (row_ptr as little-endian int64, col and the rank map
as little-endian int32), and for the 13 x 13 grid of Section 5.1 the block
count, per-shift counts (Eq. 5) and work of rank (0, 0) and of the rank
with the most tasks.

Usage: python tests/golden/make_rmat_fixture.py --scale 26 [--seed 1] [--threads 8]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402

sys.path.insert(0, os.path.dirname(HERE))
from grid_tasks import rank_tasks  # noqa: E402


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, required=True)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--q", type=int, default=13)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    n = 1 << a.scale
    t0 = time.time()
    src, dst = graphgen.rmat(a.scale, edge_factor=a.edge_factor, seed=a.seed, threads=a.threads)
    m_raw = len(src)
    print("generated %d pairs (%.0f s)" % (m_raw, time.time() - t0), flush=True)
    U = oracle.preprocess(src, dst, n)
    del src, dst
    U.lo = U.hi = None
    print("oracle preprocessing done, m = %d (%.0f s)" % (U.m, time.time() - t0), flush=True)
    T = oracle.count(U, threads=a.threads)
    print("T = %d (%.0f s)" % (T, time.time() - t0), flush=True)
    w = oracle.wedges(U)
    q = a.q
    tasks = rank_tasks(U.row_ptr, U.col, q)
    x, y = (int(v) for v in np.unravel_index(int(np.argmax(tasks)), tasks.shape))
    blocks = []
    for bx, by in ((0, 0), (x, y)):
        b, shifts = oracle.block_count_one(U, q, bx, by)
        bw = oracle.block_work(U, q, bx, by)
        blocks.append({"x": bx, "y": by, "count": b, "per_shift": [int(v) for v in shifts],
                       "tasks": bw["tasks"], "probes": bw["probes"]})
        assert bw["tasks"] == int(tasks[bx, by])
    out = {
        "workload": "rmat%d_ef%d" % (a.scale, a.edge_factor), "scale": a.scale, "seed": a.seed,
        "edge_factor": a.edge_factor, "n": n, "m_raw": m_raw, "m": U.m, "triangles": T,
        "wedges_plus": w["wedges_plus"], "probes": w["probes"], "probes_ijk": w["probes_ijk"],
        "tasks": w["tasks"], "max_out_degree": int(np.diff(U.row_ptr).max()),
        "sha256_row_ptr_i64le": digest(U.row_ptr, "<i8"), "sha256_col_i32le": digest(U.col, "<i4"),
        "sha256_rank_i32le": digest(U.rank, "<i4"),
        "grid_q": q, "grid_max_tasks_rank": [x, y], "blocks": blocks,
        "generated_by": "tests/golden/make_rmat_fixture.py --scale %d --seed %d (oracle only)"
                        % (a.scale, a.seed),
    }
    path = os.path.join(HERE, "rmat%d_seed%d.json" % (a.scale, a.seed))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote %s (%.0f s)" % (path, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
