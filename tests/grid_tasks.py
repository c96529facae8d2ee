"""Which rank of a q x q grid has the most tasks (test helper, numpy only).

Task counting here only selects which rank a test looks at; the expected
values of that rank come from the oracle (oracle.block_count_one /
oracle.block_work)."""
import numpy as np


def rank_tasks(row_ptr, col, q):
    """Tasks of every rank (x, y) of the q x q grid of Section 5.1: nonzeros
    (i, j) of U with j % q == x and i % q == y whose row i has entries after j
    and whose row j is not empty. Returns an int64 [q, q] array."""
    n = len(row_ptr) - 1
    deg = np.diff(row_ptr)
    out = np.zeros(q * q, np.int64)
    step = 1 << 22
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        p0, p1 = int(row_ptr[r0]), int(row_ptr[r1])
        if p1 == p0:
            continue
        rows = np.repeat(np.arange(r0, r1, dtype=np.int64), deg[r0:r1])
        pos = np.arange(p0, p1, dtype=np.int64)
        j = col[p0:p1].astype(np.int64)
        ok = (row_ptr[rows + 1] - pos - 1 > 0) & (deg[j] > 0)
        out += np.bincount((j % q) * q + rows % q, weights=ok, minlength=q * q).astype(np.int64)
    return out.reshape(q, q)


def max_task_rank(row_ptr, col, q):
    t = rank_tasks(row_ptr, col, q)
    x, y = np.unravel_index(int(np.argmax(t)), t.shape)
    return int(x), int(y)
