"""Seeded synthetic input graphs for the triangle-counting library.

Inputs only: this module produces raw edge lists (int32 ``src``/``dst`` pairs
that may contain duplicates, both orientations and self loops) and the
arrival/size traces of the serving workload. It holds none of the counting
method's arithmetic and is the only code the CPU oracle and the GPU path share.

The generators are written in C (``graphgen.c``) with counter-based SplitMix64
draws, so a graph depends only on its parameters and seed, never on the number
of host threads. ``build()`` compiles the shared library with gcc.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# RMAT quadrant probabilities of the Graph500 specification (a, b, c; d = 1-a-b-c).
RMAT_ABC = (0.57, 0.19, 0.19)


def build(verbose: bool = False) -> str:
    """Compile libgraphgen.so in place (gcc -O3 -fopenmp)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-parentheses",
           "-o", tmp, _SRC, "-lm"]
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
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                            i32p, i32p, ctypes.c_int]
    lib.gg_rmat.restype = ctypes.c_int
    lib.gg_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
    lib.gg_er.restype = ctypes.c_int
    lib.gg_batch_spec.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]
    lib.gg_batch_spec.restype = None
    lib.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
    lib.gg_uniform.restype = None
    lib.gg_scale_for.argtypes = [ctypes.c_int64]
    lib.gg_scale_for.restype = ctypes.c_int
    _lib = lib
    return lib


def _threads(threads):
    if threads:
        return int(threads)
    return max(1, min(16, os.cpu_count() or 1))


def scale_for(n: int) -> int:
    """Smallest s >= 1 with 2**s >= n."""
    return int(_load().gg_scale_for(int(n)))


def rmat(scale: int, edge_factor: float = 16, seed: int = 1, n: int | None = None,
         m: int | None = None, abc=RMAT_ABC, permute: bool = True, threads: int | None = None):
    """RMAT edge list: ``m`` (default ``edge_factor * 2**scale``) raw pairs on ``n``
    (default ``2**scale``) vertices. Returns int32 arrays (src, dst)."""
    lib = _load()
    if n is None:
        n = 1 << scale
    if m is None:
        m = int(round(edge_factor * n))
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = lib.gg_rmat(int(scale), int(n), int(m), int(seed), float(abc[0]), float(abc[1]),
                     float(abc[2]), int(bool(permute)), src.ctypes.data_as(i32p),
                     dst.ctypes.data_as(i32p), _threads(threads))
    if rc != 0:
        raise ValueError("gg_rmat: bad arguments scale=%d n=%d m=%d" % (scale, n, m))
    return src, dst


def er(n: int, m: int, seed: int = 1):
    """Erdos-Renyi G(n, m): m distinct unordered non-loop pairs (int32 src, dst)."""
    lib = _load()
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = lib.gg_er(int(n), int(m), int(seed), src.ctypes.data_as(i32p), dst.ctypes.data_as(i32p))
    if rc != 0:
        raise ValueError("gg_er: m=%d exceeds the pairs of n=%d" % (m, n))
    return src, dst


def er_avg_degree(n: int, avg_degree: float, seed: int = 1):
    """G(n, m) with m = round(n * avg_degree / 2)."""
    return er(n, int(round(n * avg_degree / 2.0)), seed)


def uniform(seed: int, purpose: int, count: int) -> np.ndarray:
    out = np.empty(int(count), dtype=np.float64)
    _load().gg_uniform(int(seed), int(purpose), int(count), out.ctypes.data)
    return out


@dataclass(frozen=True)
class GraphSpec:
    kind: str      # "er" or "rmat"
    n: int
    m: int         # generated pairs
    param: float   # ER average degree or RMAT edge factor
    seed: int

    def generate(self, threads: int | None = None):
        if self.kind == "er":
            return er(self.n, self.m, self.seed)
        return rmat(scale_for(self.n), seed=self.seed, n=self.n, m=self.m, threads=threads)


def generate_many(specs, threads: int = 16):
    """Edge lists of many specs, generated concurrently (the C generators run
    without the GIL); the output of each spec does not depend on threads."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(lambda s: s.generate(threads=1), specs))


def batch_specs(count: int = 4096, seed: int = 1, nmin: int = 64, nmax: int = 65536,
                er_deg=(8.0, 64.0), rmat_ef=(8.0, 32.0), seed_base: int = 1000):
    """Uneven batch: n log-uniform in [nmin, nmax]; even index ER with average
    degree U[er_deg], odd index RMAT with edge factor U[rmat_ef]; graph g uses
    seed seed_base + g."""
    lib = _load()
    kind = np.empty(count, np.int32)
    n = np.empty(count, np.int64)
    m = np.empty(count, np.int64)
    param = np.empty(count, np.float64)
    gseed = np.empty(count, np.uint64)
    lib.gg_batch_spec(int(count), int(seed), int(nmin), int(nmax), float(er_deg[0]), float(er_deg[1]),
                      float(rmat_ef[0]), float(rmat_ef[1]), int(seed_base), kind.ctypes.data,
                      n.ctypes.data, m.ctypes.data, param.ctypes.data, gseed.ctypes.data)
    return [GraphSpec("er" if kind[g] == 0 else "rmat", int(n[g]), int(m[g]), float(param[g]),
                      int(gseed[g])) for g in range(count)]


@dataclass(frozen=True)
class Request:
    index: int
    arrival_s: float
    op: str          # "count" or "support"
    spec: GraphSpec
    requery: int     # index of an earlier request whose graph is asked again, or -1


def serving_trace(num: int, rate_per_s: float, seed: int = 7, median_log2n: float = 14.0,
                  sigma: float = 1.0, nmin: int = 64, nmax: int = 1 << 22,
                  requery_frac: float = 0.3, max_rmat_scale: int = 22):
    """Poisson arrivals at ``rate_per_s``; ln n ~ N(ln 2**median_log2n, sigma) clipped to
    [nmin, nmax]; 50/50 ER (avg degree 16) / RMAT (edge factor 16); 50/50 count/support;
    a fraction ``requery_frac`` of requests re-ask an earlier request's graph."""
    u = uniform(seed, 1, 6 * num).reshape(num, 6)
    t = 0.0
    out = []
    for i in range(num):
        t += -math.log(1.0 - u[i, 0]) / rate_per_s
        op = "count" if u[i, 1] < 0.5 else "support"
        if i > 0 and u[i, 2] < requery_frac:
            j = int(u[i, 3] * i)
            out.append(Request(i, t, op, out[j].spec, j if out[j].requery < 0 else out[j].requery))
            continue
        # Box-Muller normal from two uniforms
        z = math.sqrt(-2.0 * math.log(1.0 - u[i, 3])) * math.cos(2.0 * math.pi * u[i, 4])
        n = int(round(math.exp(math.log(2.0 ** median_log2n) + sigma * z)))
        n = max(nmin, min(nmax, n))
        if u[i, 5] < 0.5:
            spec = GraphSpec("er", n, int(round(n * 16 / 2.0)), 16.0, 100000 + i)
        else:
            if scale_for(n) > max_rmat_scale:
                n = 1 << max_rmat_scale
            spec = GraphSpec("rmat", n, 16 * n, 16.0, 100000 + i)
        out.append(Request(i, t, op, spec, -1))
    return out
