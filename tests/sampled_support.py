"""Exact full support of sampled edges of a large graph (test helper, CPU).

Full support of an edge {a, b} is the number of triangles containing it, i.e.
|Adj(a) & Adj(b)| in the simple graph (Section 2). For a few sampled edges of
U (rank space, every entry of row a greater than a) the helper builds Adj(v)
of just the vertices involved: the upper part is U's row v, the lower part
the rows whose entries include v, found in one vectorised scan of U's column
array. Nothing here is shared with the GPU path.
"""
import numpy as np


def sampled_full_support(row_ptr: np.ndarray, col: np.ndarray, positions: np.ndarray) -> np.ndarray:
    """Full support of the U entries at `positions` (int64 array), in order."""
    positions = np.asarray(positions, dtype=np.int64)
    n = len(row_ptr) - 1
    # the row (lower endpoint) of each sampled entry
    rows = np.searchsorted(row_ptr, positions, side="right") - 1
    cols = col[positions].astype(np.int64)
    verts = np.unique(np.concatenate([rows, cols]))
    # lower neighbours of the sampled vertices: rows a with v in U_a
    mask = np.zeros(n, dtype=bool)
    mask[verts] = True
    hit = np.nonzero(mask[col])[0]
    hit_rows = np.searchsorted(row_ptr, hit, side="right") - 1
    hit_cols = col[hit]
    order = np.argsort(hit_cols, kind="stable")
    hit_cols = hit_cols[order]
    hit_rows = hit_rows[order]
    lower = {}
    starts = np.searchsorted(hit_cols, verts, side="left")
    ends = np.searchsorted(hit_cols, verts, side="right")
    for v, s, e in zip(verts.tolist(), starts.tolist(), ends.tolist()):
        lower[v] = hit_rows[s:e]

    def adj(v):
        return np.concatenate([lower[v], col[row_ptr[v]:row_ptr[v + 1]].astype(np.int64)])

    cache = {}
    out = np.empty(len(positions), dtype=np.int64)
    for i, (a, b) in enumerate(zip(rows.tolist(), cols.tolist())):
        for v in (a, b):
            if v not in cache:
                cache[v] = np.unique(adj(v))
        out[i] = len(np.intersect1d(cache[a], cache[b], assume_unique=True))
    return out


def sample_positions(row_ptr: np.ndarray, seed: int, uniform: int = 1024, top_rows: int = 16,
                     per_row: int = 64) -> np.ndarray:
    """Entries of U to check: `uniform` positions drawn uniformly, plus up to
    `per_row` entries (evenly spaced) of each of the `top_rows` longest rows,
    whose tables are the largest ones in the count kernels."""
    m = int(row_ptr[-1])
    if m == 0:
        return np.zeros(0, dtype=np.int64)
    rng = np.random.default_rng(seed)
    picks = [rng.integers(0, m, min(uniform, m))]
    lens = np.diff(row_ptr)
    for r in np.argsort(lens, kind="stable")[::-1][:top_rows]:
        d = int(lens[r])
        if d == 0:
            continue
        k = min(per_row, d)
        picks.append(int(row_ptr[r]) + np.linspace(0, d - 1, k).astype(np.int64))
    return np.unique(np.concatenate(picks))
