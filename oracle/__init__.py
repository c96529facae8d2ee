"""CPU oracle for exact triangle counting (Tom and Karypis, ICPP 2019).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check and
by the benchmark's CPU-baseline leg, never by the library's product path. It
shares no code with the GPU path; only the seeded input generator
(``graphgen``) serves both.

Two layers:

* ``oracle.c`` (plain C, qsort as the only primitive, OpenMP only across the
  independent rows of Eq. 2's sum) - follows the paper's definitions in order;
  see its header for the passage each function follows.
* ``brute_*`` (pure Python sets and loops, for graphs of a few hundred
  vertices) - the definitions of Section 2 written out with no ordering at
  all, used to pin the C layer.

Parity status: each function is pinned in ``tests/test_oracle.py`` (and the
property tests in ``tests/test_oracle_properties.py``) by something other
than itself: closed forms, brute force over vertex triples or edge subsets,
trace(A^3), or identities between independent functions (row-range sums
against the total, per-rank work against the whole graph's). The pins of
each function are listed in ``PINS`` below; a function missing from it would
be "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MODE_FULL = 0
MODE_ORIENTED = 1


def build(verbose: bool = False) -> str:
    """Compile liboracle.so in place (gcc -O2 -fopenmp)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oc_simple_edges.argtypes = [P, P, I64, I64, P, P]
    lib.oc_simple_edges.restype = I64
    lib.oc_degree_order.argtypes = [P, P, I64, I64, P, P]
    lib.oc_degree_order.restype = ctypes.c_int
    lib.oc_build_upper.argtypes = [P, P, I64, I64, P, P, P]
    lib.oc_build_upper.restype = ctypes.c_int
    lib.oc_count.argtypes = [P, P, I64, ctypes.c_int]
    lib.oc_count.restype = I64
    lib.oc_count_rows.argtypes = [P, P, I64, I64, ctypes.c_int]
    lib.oc_count_rows.restype = I64
    lib.oc_support.argtypes = [P, P, I64, ctypes.c_int, P]
    lib.oc_support.restype = I64
    lib.oc_wedges.argtypes = [P, P, I64, P]
    lib.oc_wedges.restype = None
    lib.oc_block_counts.argtypes = [P, P, I64, I64, P, P]
    lib.oc_block_counts.restype = None
    lib.oc_block_count_one.argtypes = [P, P, I64, I64, I64, I64, P]
    lib.oc_block_count_one.restype = I64
    lib.oc_pair_common.argtypes = [P, P, I64, I64]
    lib.oc_pair_common.restype = I64
    lib.oc_build_adjacency.argtypes = [P, P, I64, I64, P, P]
    lib.oc_build_adjacency.restype = ctypes.c_int
    lib.oc_block_work.argtypes = [P, P, I64, I64, I64, I64, P]
    lib.oc_block_work.restype = ctypes.c_int
    lib.oc_vertex_triangles.argtypes = [P, P, I64, P]
    lib.oc_vertex_triangles.restype = I64
    lib.oc_truss.argtypes = [P, P, I64, P]
    lib.oc_truss.restype = I64
    lib.oc_max_threads.argtypes = []
    lib.oc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ok(rc):
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    return rc


def max_threads() -> int:
    return int(_load().oc_max_threads())


@dataclass
class Upper:
    """The oracle's preprocessed graph: simple edges (original ids), degrees,
    rank (perm[orig] = rank) and the upper-triangular CSR in rank space."""
    n: int
    lo: np.ndarray
    hi: np.ndarray
    deg: np.ndarray
    rank: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])


def simple_edges(src, dst, n):
    lib = _load()
    src = _c(src, np.int32)
    dst = _c(dst, np.int32)
    m_raw = len(src)
    lo = np.empty(max(m_raw, 1), np.int32)
    hi = np.empty(max(m_raw, 1), np.int32)
    m = lib.oc_simple_edges(src.ctypes.data, dst.ctypes.data, m_raw, int(n), lo.ctypes.data,
                            hi.ctypes.data)
    if m == -1:
        raise ValueError("vertex id out of range [0, n)")
    if m < 0:
        raise MemoryError("oracle allocation failed")
    return lo[:m].copy(), hi[:m].copy()


def preprocess(src, dst, n) -> Upper:
    """Simple graph -> degree order -> upper CSR (Sections 2, 3.1, 5.3)."""
    lib = _load()
    lo, hi = simple_edges(src, dst, n)
    m = len(lo)
    deg = np.empty(max(n, 1), np.int32)
    rank = np.empty(max(n, 1), np.int32)
    _ok(lib.oc_degree_order(lo.ctypes.data, hi.ctypes.data, m, int(n), deg.ctypes.data,
                            rank.ctypes.data))
    row_ptr = np.empty(n + 1, np.int64)
    col = np.empty(max(m, 1), np.int32)
    _ok(lib.oc_build_upper(lo.ctypes.data, hi.ctypes.data, m, int(n), rank.ctypes.data,
                           row_ptr.ctypes.data, col.ctypes.data))
    return Upper(int(n), lo, hi, deg[:n], rank[:n], row_ptr, col[:m])


def count(U: Upper, threads: int | None = None) -> int:
    """Eq. 2 total by list-based intersection."""
    return int(_load().oc_count(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n,
                                int(threads or max_threads())))


def count_rows(U: Upper, a_lo: int, a_hi: int, threads: int | None = None) -> int:
    """Eq. 2's sum over the rows a of U in [a_lo, a_hi) only."""
    return int(_load().oc_count_rows(U.row_ptr.ctypes.data, U.col.ctypes.data, int(a_lo),
                                     int(a_hi), int(threads or max_threads())))


def support(U: Upper, mode: int = MODE_FULL):
    """(T, per-edge int32 values in U order). mode FULL: triangles per edge;
    ORIENTED: c(a, b) of Eq. 1."""
    s = np.empty(max(U.m, 1), np.int32)
    T = _load().oc_support(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, int(mode), s.ctypes.data)
    return int(T), s[:U.m]


def wedges(U: Upper) -> dict:
    out = np.zeros(4, np.int64)
    _load().oc_wedges(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, out.ctypes.data)
    return {"wedges_plus": int(out[0]), "probes": int(out[1]), "probes_ijk": int(out[2]),
            "tasks": int(out[3])}


def block_counts(U: Upper, q: int):
    """(B[q, q], per_shift[q, q, q]) under the C[L] convention of Section 5.1."""
    B = np.zeros(q * q, np.int64)
    S = np.zeros(q * q * q, np.int64)
    _load().oc_block_counts(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, int(q), B.ctypes.data,
                            S.ctypes.data)
    return B.reshape(q, q), S.reshape(q, q, q)


def block_count_one(U: Upper, q: int, x: int, y: int):
    """(B[x][y], per_shift[q]) for rank (x, y) alone (Section 5.1, Eq. 5)."""
    S = np.zeros(q, np.int64)
    B = _load().oc_block_count_one(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, int(q), int(x), int(y),
                                   S.ctypes.data)
    return int(B), S


@dataclass
class Adjacency:
    n: int
    ptr: np.ndarray
    adj: np.ndarray

    def common(self, u: int, v: int) -> int:
        return int(_load().oc_pair_common(self.ptr.ctypes.data, self.adj.ctypes.data, int(u), int(v)))


def adjacency(lo, hi, n) -> Adjacency:
    lo = _c(lo, np.int32)
    hi = _c(hi, np.int32)
    m = len(lo)
    ptr = np.empty(n + 1, np.int64)
    adj = np.empty(max(2 * m, 1), np.int32)
    _ok(_load().oc_build_adjacency(lo.ctypes.data, hi.ctypes.data, m, int(n), ptr.ctypes.data,
                                   adj.ctypes.data))
    return Adjacency(int(n), ptr, adj[:2 * m])


def block_work(U: Upper, q: int, x: int, y: int) -> dict:
    """Work of rank (x, y) of the q x q grid (Section 5.1; Section 7.2's
    balance and intersection-count tables): tasks, probes, probes per shift
    (closing vertex in the shift's residue class, Eq. 5) and the tasks each
    shift would intersect (probe list and hashed list both hold an entry of
    that class)."""
    out = np.zeros(2 + 2 * q, np.int64)
    _ok(_load().oc_block_work(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, int(q), int(x), int(y),
                              out.ctypes.data))
    return {"tasks": int(out[0]), "probes": int(out[1]), "shift_probes": out[2:2 + q].copy(),
            "shift_tasks": out[2 + q:].copy()}


def vertex_triangles(U: Upper) -> np.ndarray:
    """t[v] = triangles containing original vertex v (int64[n])."""
    t = np.zeros(max(U.n, 1), np.int64)
    _load().oc_vertex_triangles(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, t.ctypes.data)
    return t[U.rank]


def clustering(U: Upper):
    """Local clustering coefficients and transitivity from per-vertex
    triangle counts (Section 1's application): cc[v] = t(v) / C(d(v), 2) in
    float64 (0 where d(v) < 2), transitivity = 3 T / sum_v C(d(v), 2) (0 if
    there is no pair of adjacent edges). Both are one division of two exact
    integers, so they are correctly rounded."""
    t = vertex_triangles(U)
    d = U.deg.astype(np.int64)
    pairs = d * (d - 1) // 2
    cc = np.zeros(U.n, np.float64)
    nz = pairs > 0
    cc[nz] = t[nz].astype(np.float64) / pairs[nz].astype(np.float64)
    W = int(pairs.sum())
    T3 = int(t.sum())  # = 3 T
    return cc, (float(T3) / float(W) if W else 0.0), t, W


def truss(U: Upper):
    """(largest trussness, int32 trussness of every edge in U order)."""
    tau = np.zeros(max(U.m, 1), np.int32)
    kmax = _ok(_load().oc_truss(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n, tau.ctypes.data))
    return int(kmax), tau[:U.m]


# ---------------------------------------------------------------------------
# Pure-Python brute force (Section 2's definitions, no ordering), small graphs.
# ---------------------------------------------------------------------------

def brute_edge_set(src, dst):
    """The simple undirected graph as a set of frozensets {u, v}, u != v."""
    return {frozenset((int(u), int(v))) for u, v in zip(src, dst) if int(u) != int(v)}


def brute_count(src, dst, n) -> int:
    """Number of 3-vertex sets whose three pairs are all edges (O(n^3))."""
    E = brute_edge_set(src, dst)
    adj = [set() for _ in range(n)]
    for e in E:
        u, v = tuple(e)
        adj[u].add(v)
        adj[v].add(u)
    t = 0
    for i in range(n):
        for j in range(i + 1, n):
            if j not in adj[i]:
                continue
            for k in range(j + 1, n):
                if k in adj[i] and k in adj[j]:
                    t += 1
    return t


def brute_edge_support(src, dst, n) -> dict:
    """{frozenset({u, v}): number of triangles containing the edge}."""
    E = brute_edge_set(src, dst)
    adj = [set() for _ in range(n)]
    for e in E:
        u, v = tuple(e)
        adj[u].add(v)
        adj[v].add(u)
    return {e: sum(1 for w in range(n) if all(w in adj[x] for x in e)) for e in E}


# The CPU tests that pin each function against something other than itself
# (closed forms, brute force, independent identities).
PINS = {
    "simple_edges": ["test_preprocess_structure", "test_count_is_the_triple_definition"],
    "preprocess": ["test_preprocess_structure", "test_preprocess_idempotent_on_simple_input",
                   "test_out_of_range_rejected", "test_oriented_support_is_eq1"],
    "count": ["test_closed_forms", "test_brute_force_random", "test_trace_a_cubed",
              "test_count_is_the_triple_definition", "test_relabel_duplicate_and_loop_invariance"],
    "count_rows": ["test_count_rows_partition_sums_to_total", "test_count_rows_single_row_is_eq1_by_sets",
                   "test_count_rows_empty_and_closed_form", "test_count_rows_equals_oriented_support_row_sums"],
    "support": ["test_support_complete", "test_support_wheel_and_friendship", "test_support_tripartite",
                "test_support_brute", "test_full_support_is_triangles_per_edge", "test_oriented_support_is_eq1"],
    "wedges": ["test_wedges_brute"],
    "block_counts": ["test_block_counts", "test_blocks_and_shifts_decompose_T"],
    "block_count_one": ["test_block_counts", "test_blocks_and_shifts_decompose_T"],
    "block_work": ["test_block_work_sums_over_ranks", "test_block_work_by_sets"],
    "adjacency": ["test_pair_common_matches_support"],
    "vertex_triangles": ["test_vertex_triangles_closed_forms", "test_vertex_triangles_diagonal_of_a_cubed",
                         "test_vertex_triangles_are_triangles_through_each_vertex"],
    "clustering": ["test_clustering_closed_forms", "test_transitivity_matches_counts"],
    "truss": ["test_truss_closed_forms", "test_truss_brute_force_over_subsets", "test_truss_invariants_rmat",
              "test_truss_is_the_subset_definition"],
    "brute_edge_set": ["test_er_simple", "test_preprocess_structure"],
    "brute_count": ["test_closed_forms_brute"],
    "brute_edge_support": ["test_support_brute_closed_forms"],
}
