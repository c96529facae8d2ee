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

Parity status: every function here is pinned by closed forms, brute force or
invariants in ``tests/test_oracle.py``; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import itertools
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
    lib.oc_degree_order.restype = None
    lib.oc_build_upper.argtypes = [P, P, I64, I64, P, P, P]
    lib.oc_build_upper.restype = None
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
    lib.oc_build_adjacency.restype = None
    lib.oc_max_threads.argtypes = []
    lib.oc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


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
    lib.oc_degree_order(lo.ctypes.data, hi.ctypes.data, m, int(n), deg.ctypes.data, rank.ctypes.data)
    row_ptr = np.empty(n + 1, np.int64)
    col = np.empty(max(m, 1), np.int32)
    lib.oc_build_upper(lo.ctypes.data, hi.ctypes.data, m, int(n), rank.ctypes.data,
                       row_ptr.ctypes.data, col.ctypes.data)
    return Upper(int(n), lo, hi, deg[:n], rank[:n], row_ptr, col[:m])


def count(U: Upper, threads: int | None = None) -> int:
    """Eq. 2 total by list-based intersection."""
    return int(_load().oc_count(U.row_ptr.ctypes.data, U.col.ctypes.data, U.n,
                                int(threads or max_threads())))


def count_rows(U: Upper, a_lo: int, a_hi: int, threads: int | None = None) -> int:
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
    _load().oc_build_adjacency(lo.ctypes.data, hi.ctypes.data, m, int(n), ptr.ctypes.data,
                               adj.ctypes.data)
    return Adjacency(int(n), ptr, adj[:2 * m])


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


def brute_triangles(src, dst, n):
    """All triangles as sorted vertex triples (original ids)."""
    E = brute_edge_set(src, dst)
    out = []
    for i, j, k in itertools.combinations(range(n), 3):
        if frozenset((i, j)) in E and frozenset((i, k)) in E and frozenset((j, k)) in E:
            out.append((i, j, k))
    return out
