"""Exact triangle counting on AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libtc.so`` (the C ABI declared in ``include/tc.h``).
Every step of the path runs in the library's HIP kernels; this module only
marshals arguments: torch tensors on a ROCm device provide the memory
(``data_ptr()``) and ``torch.cuda`` streams the ordering. There is no CPU
fallback: importing the package without a built ``libtc.so`` raises.

Functions carry the C names: tc_preprocess, tc_graph_info, tc_graph_export,
tc_count, tc_edge_support, tc_block_count, tc_batch_create, tc_batch_count,
tc_batch_free, tc_batch_describe, tc_count_batched, tc_batch_autotune, tc_graph_free.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "TCError", "Graph", "Batch", "tc_preprocess", "tc_graph_info", "tc_graph_export", "tc_count",
    "tc_edge_support", "tc_block_count", "tc_batch_create", "tc_batch_count", "tc_batch_free",
    "tc_batch_describe", "tc_batch_autotune", "tc_count_batched", "tc_count_batched_noalloc", "Server", "tc_release_cached_memory",
    "tc_memory_stats", "tc_graph_free", "tc_graph_class_stats", "tc_vertex_triangles", "tc_clustering",
    "tc_transitivity", "tc_truss", "tc_graph_variant", "tc_block_stats", "TC_VARIANT_IJK", "TC_VARIANT_NO_DCSR",
    "TC_VARIANT_MUL_HASH", "Timer", "TC_SUPPORT_FULL", "tc_graph_retune", "tc_graph_work_params",
    "tc_graph_autotune", "tc_tuning_load", "tc_tuning_save", "tc_tuning_get", "tc_tuning_set", "tc_tuning_key",
    "TC_SUPPORT_ORIENTED", "TC_NUM_CLASSES", "library_path",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libtc.so")

TC_OK, TC_EINVAL, TC_ENOMEM, TC_EDEVICE, TC_EOVERFLOW, TC_EBUSY, TC_ECANCELED = range(7)
TC_SUPPORT_FULL = 0
TC_SUPPORT_ORIENTED = 1
TC_NUM_CLASSES = 7

if not os.path.exists(library_path):
    raise ImportError(
        "libtc.so is not built at %s; run `python paper_1907_09575_amd/build.py` "
        "(or __graft_entry__.build())" % library_path)

_lib = ctypes.CDLL(library_path)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


class _Info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "m_raw", "m", "wedges_plus", "probes", "tasks", "max_out_degree", "device_bytes")]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("tc_preprocess", [_P, _P, _I64, _I32, _P, ctypes.POINTER(_P)])
_sig("tc_graph_info", [_P, ctypes.POINTER(_Info)])
_sig("tc_graph_export", [_P, _P, _P, _P, _P])
_sig("tc_count", [_P, _P, _P])
_sig("tc_edge_support", [_P, ctypes.c_int, _P, _P, _P])
_sig("tc_block_count", [_P, _I32, _I32, _I32, _P, _P, _P])
_sig("tc_batch_create", [ctypes.POINTER(_P), _I32, ctypes.c_char_p, _P, ctypes.POINTER(_P)])
_sig("tc_batch_count", [_P, _P, _P])
_sig("tc_batch_free", [_P], None)
_sig("tc_count_batched", [ctypes.POINTER(_P), _I32, _P, ctypes.c_char_p, _P])
_sig("tc_count_batched_noalloc", [ctypes.POINTER(_P), _I32, _P, _P])
_sig("tc_batch_describe", [_P, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_batch_autotune", [ctypes.POINTER(_P), _I32, _P, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_graph_free", [_P], None)
_sig("tc_vertex_triangles", [_P, _P, _P])
_sig("tc_graph_variant", [_P, _I32, _P, ctypes.POINTER(_P)])
_sig("tc_block_stats", [_P, _I32, _I32, _I32, _P, _P])
_sig("tc_clustering", [_P, _P, _P, _P, _P])
_sig("tc_transitivity", [_P, ctypes.POINTER(ctypes.c_double), _P])
_sig("tc_truss", [_P, _P, ctypes.POINTER(_I32), _P])
_sig("tc_graph_class_stats", [_P, _P])
_sig("tc_tuning_load", [ctypes.c_char_p])
_sig("tc_tuning_save", [ctypes.c_char_p])
_sig("tc_tuning_get", [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_tuning_set", [ctypes.c_char_p, ctypes.c_char_p])
_sig("tc_tuning_key", [ctypes.c_char_p, _I64, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_graph_retune", [_P, ctypes.c_char_p, _P, ctypes.POINTER(_P)])
_sig("tc_graph_work_params", [_P, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_graph_autotune", [_P, _P, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_class_name", [_I32], ctypes.c_char_p)
_sig("tc_timer_create", [_I32, ctypes.POINTER(_P)])
_sig("tc_timer_attach", [_P])
_sig("tc_timer_summary", [_P, ctypes.c_char_p, _I64])
_sig("tc_timer_reset", [_P])
_sig("tc_timer_free", [_P], None)
_sig("tc_status_string", [ctypes.c_int], ctypes.c_char_p)
_sig("tc_last_error", [], ctypes.c_char_p)
_sig("tc_version", [], ctypes.c_char_p)


class TCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.tc_last_error().decode() or _lib.tc_status_string(status).decode()
        super().__init__("%s failed: %s [%s]" % (where, msg, _lib.tc_status_string(status).decode()))


def _check(status: int, where: str):
    if status != TC_OK:
        raise TCError(status, where)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev_ptr(t: torch.Tensor | None, dtype, what: str, numel: int | None = None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s needs %d elements, has %d" % (what, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return _lib.tc_version().decode()


class Graph:
    """Owning wrapper of a tc_graph handle (freed with the object)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        self._info = None

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph already freed")
        return self._h

    def info(self) -> dict:
        if self._info is None:
            self._info = tc_graph_info(self)
        return self._info

    @property
    def n(self) -> int:
        return self.info()["n"]

    @property
    def m(self) -> int:
        return self.info()["m"]

    def free(self):
        if self._h:
            _lib.tc_graph_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def tc_preprocess(src: torch.Tensor, dst: torch.Tensor, n: int, stream=None) -> Graph:
    """Build the device-resident graph from int32 device edge arrays."""
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    out = ctypes.c_void_p()
    _check(_lib.tc_preprocess(_dev_ptr(src, torch.int32, "src"), _dev_ptr(dst, torch.int32, "dst"),
                                   src.numel(), int(n), _stream(stream), ctypes.byref(out)),
                "tc_preprocess")
    return Graph(out.value)


def tc_graph_info(g: Graph) -> dict:
    info = _Info()
    _check(_lib.tc_graph_info(g.handle, ctypes.byref(info)), "tc_graph_info")
    return {name: int(getattr(info, name)) for name, _ in _Info._fields_}


def tc_graph_export(g: Graph, row_ptr=None, col=None, perm=None, stream=None):
    """Copy U and the relabelling into device tensors (allocated if None)."""
    info = g.info()
    dev = torch.device("cuda", torch.cuda.current_device())
    if row_ptr is None:
        row_ptr = torch.empty(info["n"] + 1, dtype=torch.int64, device=dev)
    if col is None:
        col = torch.empty(max(info["m"], 1), dtype=torch.int32, device=dev)
    if perm is None:
        perm = torch.empty(info["n"], dtype=torch.int32, device=dev)
    _check(_lib.tc_graph_export(g.handle, _dev_ptr(row_ptr, torch.int64, "row_ptr", info["n"] + 1),
                                _dev_ptr(col, torch.int32, "col", info["m"]),
                                _dev_ptr(perm, torch.int32, "perm", info["n"]), _stream(stream)),
           "tc_graph_export")
    return row_ptr, col[:info["m"]], perm


def _count_out(out):
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=torch.device("cuda", torch.cuda.current_device()))
    return out


def tc_count(g: Graph, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Triangle count into a 1-element int64 device tensor (asynchronous)."""
    out = _count_out(out)
    _check(_lib.tc_count(g.handle, _dev_ptr(out, torch.int64, "count", 1), _stream(stream)), "tc_count")
    return out


def tc_edge_support(g: Graph, mode: int = TC_SUPPORT_FULL, support: torch.Tensor | None = None,
                    count: torch.Tensor | None = None, stream=None):
    """Per-edge support (int32, U order) and optionally the total."""
    m = g.info()["m"]
    if support is None:
        support = torch.empty(max(m, 1), dtype=torch.int32,
                              device=torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.tc_edge_support(g.handle, int(mode), _dev_ptr(support, torch.int32, "support", m),
                                _dev_ptr(count, torch.int64, "count", 1), _stream(stream)),
           "tc_edge_support")
    return support[:m], count


def tc_block_count(g: Graph, q: int, x: int, y: int, count: torch.Tensor | None = None,
                   per_shift: torch.Tensor | None = None, stream=None):
    """One rank's block of the q x q cyclic decomposition (count, per-shift)."""
    count = _count_out(count)
    _check(_lib.tc_block_count(g.handle, int(q), int(x), int(y), _dev_ptr(count, torch.int64, "count", 1),
                               _dev_ptr(per_shift, torch.int64, "per_shift", int(q)), _stream(stream)),
           "tc_block_count")
    return count, per_shift


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


TC_VARIANT_IJK, TC_VARIANT_NO_DCSR, TC_VARIANT_MUL_HASH = 1, 2, 4


def tc_graph_variant(g: Graph, flags: int, stream=None) -> Graph:
    """A handle counting g's triangles with Section 5.2's optimizations
    undone (TC_VARIANT_* flags); it shares g's U, so keep g alive."""
    out = ctypes.c_void_p()
    _check(_lib.tc_graph_variant(g.handle, int(flags), _stream(stream), ctypes.byref(out)), "tc_graph_variant")
    v = Graph(out.value)
    v.base = g  # keeps the shared arrays' owner alive
    return v


def tc_graph_retune(g: Graph, params=None, stream=None) -> Graph:
    """A handle counting g with its work cut by other row-bucket thresholds
    (dict or JSON text with heavy_min, pack_target, pack_slots, wave_chunk);
    it shares g's U, so keep g alive."""
    out = ctypes.c_void_p()
    _check(_lib.tc_graph_retune(g.handle, _tuning(params), _stream(stream), ctypes.byref(out)), "tc_graph_retune")
    v = Graph(out.value)
    v.base = g
    return v


def tc_graph_work_params(g: Graph) -> dict:
    """The row-bucket thresholds g's work was cut with."""
    import json
    buf = ctypes.create_string_buffer(512)
    _check(_lib.tc_graph_work_params(g.handle, buf, len(buf)), "tc_graph_work_params")
    return json.loads(buf.value.decode())


def tc_graph_autotune(g: Graph, stream=None) -> dict:
    """Time tc_count under candidate thresholds; the best goes into the
    tuning table for graphs of g's size: {"key", "best", "candidates"}."""
    import json
    buf = ctypes.create_string_buffer(1 << 14)
    _check(_lib.tc_graph_autotune(g.handle, _stream(stream), buf, len(buf)), "tc_graph_autotune")
    return json.loads(buf.value.decode())


def tc_tuning_load(path: str):
    _check(_lib.tc_tuning_load(os.fsencode(path)), "tc_tuning_load")


def tc_tuning_save(path: str):
    _check(_lib.tc_tuning_save(os.fsencode(path)), "tc_tuning_save")


def tc_tuning_get(key: str) -> dict | None:
    """The tuning-table entry a lookup of key finds (None if there is none)."""
    import json
    buf = ctypes.create_string_buffer(4096)
    _check(_lib.tc_tuning_get(key.encode(), buf, len(buf)), "tc_tuning_get")
    return json.loads(buf.value.decode()) if buf.value else None


def tc_tuning_set(key: str, entry=None):
    """Set (dict or JSON text) or remove (None) a tuning-table entry."""
    _check(_lib.tc_tuning_set(key.encode(), _tuning(entry)), "tc_tuning_set")


def tc_tuning_key(kind: str, edges: int) -> str:
    buf = ctypes.create_string_buffer(256)
    _check(_lib.tc_tuning_key(kind.encode(), int(edges), buf, len(buf)), "tc_tuning_key")
    return buf.value.decode()


def tc_vertex_triangles(g: Graph, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Triangles through every vertex (int64, original ids)."""
    n = g.info()["n"]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=_dev())
    _check(_lib.tc_vertex_triangles(g.handle, _dev_ptr(out, torch.int64, "tri", n), _stream(stream)),
           "tc_vertex_triangles")
    return out


def tc_clustering(g: Graph, cc: torch.Tensor | None = None, tri: torch.Tensor | None = None,
                  sums: torch.Tensor | None = None, stream=None):
    """Local clustering coefficients (float64, original ids); optionally the
    per-vertex triangles and [3T, sum C(d, 2)]."""
    n = g.info()["n"]
    if cc is None:
        cc = torch.empty(n, dtype=torch.float64, device=_dev())
    _check(_lib.tc_clustering(g.handle, _dev_ptr(cc, torch.float64, "cc", n), _dev_ptr(tri, torch.int64, "tri", n),
                              _dev_ptr(sums, torch.int64, "sums", 2), _stream(stream)), "tc_clustering")
    return cc, tri, sums


def tc_transitivity(g: Graph, stream=None) -> float:
    out = ctypes.c_double()
    _check(_lib.tc_transitivity(g.handle, ctypes.byref(out), _stream(stream)), "tc_transitivity")
    return out.value


def tc_truss(g: Graph, tau: torch.Tensor | None = None, stream=None):
    """(trussness int32 in U order, largest trussness)."""
    m = g.info()["m"]
    if tau is None:
        tau = torch.empty(max(m, 1), dtype=torch.int32, device=_dev())
    k = _I32()
    _check(_lib.tc_truss(g.handle, _dev_ptr(tau, torch.int32, "tau", m), ctypes.byref(k), _stream(stream)),
           "tc_truss")
    return tau[:m], k.value


def tc_block_stats(g: Graph, q: int, x: int, y: int, out: torch.Tensor | None = None, stream=None):
    """Work of rank (x, y) of the q x q grid: int64 device tensor
    [tasks, probes, shift_probes[q], shift_tasks[q]]."""
    if out is None:
        out = torch.empty(2 + 2 * int(q), dtype=torch.int64, device=_dev())
    _check(_lib.tc_block_stats(g.handle, int(q), int(x), int(y), _dev_ptr(out, torch.int64, "out", 2 + 2 * int(q)),
                               _stream(stream)), "tc_block_stats")
    return out


class Batch:
    """Owning wrapper of a tc_batch plan; keeps its graphs alive."""

    def __init__(self, handle: int, graphs):
        self._h = ctypes.c_void_p(handle)
        self.graphs = list(graphs)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("batch already freed")
        return self._h

    def free(self):
        if self._h:
            _lib.tc_batch_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _handles(graphs):
    arr = (ctypes.c_void_p * max(len(graphs), 1))()
    for i, g in enumerate(graphs):
        arr[i] = g.handle.value
    return arr


def _tuning(tuning):
    if tuning is None:
        return None
    if isinstance(tuning, (bytes, str)):
        return tuning.encode() if isinstance(tuning, str) else tuning
    import json
    return json.dumps(tuning).encode()


def tc_batch_create(graphs, tuning=None, stream=None) -> Batch:
    out = ctypes.c_void_p()
    _check(_lib.tc_batch_create(_handles(graphs), len(graphs), _tuning(tuning), _stream(stream),
                                ctypes.byref(out)), "tc_batch_create")
    return Batch(out.value, graphs)


def tc_batch_count(plan: Batch, counts: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if counts is None:
        counts = torch.empty(max(len(plan.graphs), 1), dtype=torch.int64,
                             device=torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.tc_batch_count(plan.handle, _dev_ptr(counts, torch.int64, "counts", len(plan.graphs)),
                               _stream(stream)), "tc_batch_count")
    return counts


def tc_batch_free(plan: Batch):
    plan.free()


def tc_batch_describe(plan: Batch) -> dict:
    """The plan's schedule and size (units, grid, LDS bytes, ...)."""
    import json
    buf = ctypes.create_string_buffer(1024)
    _check(_lib.tc_batch_describe(plan.handle, buf, len(buf)), "tc_batch_describe")
    return json.loads(buf.value.decode())


def tc_batch_autotune(graphs, stream=None) -> dict:
    """Time candidate schedules and thresholds on these graphs:
    {"key", "best", "plan", "candidates"}; "best" is stored in the tuning
    table for batches of this size."""
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.tc_batch_autotune(_handles(graphs), len(graphs), _stream(stream), buf, len(buf)),
           "tc_batch_autotune")
    return json.loads(buf.value.decode())


def tc_count_batched(graphs, counts: torch.Tensor | None = None, tuning=None, stream=None):
    if counts is None:
        counts = torch.empty(max(len(graphs), 1), dtype=torch.int64,
                             device=torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.tc_count_batched(_handles(graphs), len(graphs),
                                 _dev_ptr(counts, torch.int64, "counts", len(graphs)), _tuning(tuning),
                                 _stream(stream)), "tc_count_batched")
    return counts


def tc_count_batched_noalloc(graphs, counts: torch.Tensor, stream=None):
    """tc_count_batched without device allocation (the library's fixed
    scratch array); `counts` is a caller-allocated int64 device tensor."""
    _check(_lib.tc_count_batched_noalloc(_handles(graphs), len(graphs),
                                         _dev_ptr(counts, torch.int64, "counts", len(graphs)),
                                         _stream(stream)), "tc_count_batched_noalloc")
    return counts


class _Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("n", ctypes.c_int32), ("m_raw", ctypes.c_int64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("graph_key", ctypes.c_uint64),
                ("support_out", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cache_hit", ctypes.c_int32), ("count", ctypes.c_int64),
                ("m", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_ready", ctypes.c_double), ("t_done", ctypes.c_double)]


TC_REQ_COUNT, TC_REQ_SUPPORT_FULL, TC_REQ_SUPPORT_ORIENTED = 0, 1, 2
_OPS = {"count": TC_REQ_COUNT, "support": TC_REQ_SUPPORT_FULL, "support_full": TC_REQ_SUPPORT_FULL,
        "support_oriented": TC_REQ_SUPPORT_ORIENTED}

_sig("tc_release_cached_memory", [], None)
_sig("tc_memory_stats", [ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)])


def tc_release_cached_memory():
    """Return the library's cached device blocks to the runtime."""
    _lib.tc_release_cached_memory()


def tc_memory_stats() -> dict:
    """Device bytes the library has handed out, holds cached, and its peak."""
    a, b, c = _I64(), _I64(), _I64()
    _check(_lib.tc_memory_stats(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "tc_memory_stats")
    return {"in_use": a.value, "cached": b.value, "peak": c.value}


_sig("tc_server_create", [_I64, _I32, ctypes.c_char_p, ctypes.POINTER(_P)])
_sig("tc_server_submit", [_P, ctypes.POINTER(_Request), ctypes.POINTER(_I64)])
_sig("tc_server_poll", [_P, _I64, _I32, ctypes.POINTER(_Result)])
_sig("tc_server_cancel", [_P, _I64])
_sig("tc_server_stats", [_P, ctypes.c_char_p, ctypes.c_size_t])
_sig("tc_server_destroy", [_P], None)


class Server:
    """The served form (tc_server_*): submit count/support requests of host
    edge lists; results come back by ticket. Host arrays are kept alive here
    until their request is polled."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, options=None):
        import json
        out = ctypes.c_void_p()
        opts = None if options is None else json.dumps(options).encode()
        _check(_lib.tc_server_create(int(budget_bytes), int(max_slots), opts, ctypes.byref(out)),
               "tc_server_create")
        self._h = out
        self._keep = {}

    def submit(self, op, src, dst, n: int, key: int = 0, support_out=None) -> int:
        import numpy as np
        opc = _OPS[op] if isinstance(op, str) else int(op)
        src = None if src is None else np.ascontiguousarray(src, dtype=np.int32)
        dst = None if dst is None else np.ascontiguousarray(dst, dtype=np.int32)
        m_raw = 0 if src is None else len(src)
        if opc != TC_REQ_COUNT and support_out is None:
            support_out = np.empty(max(m_raw, 1), dtype=np.int32)
        if support_out is not None:
            assert support_out.dtype == np.int32 and support_out.flags.c_contiguous
            if src is None:
                m_raw = len(support_out)
        req = _Request(opc, int(n), int(m_raw), None if src is None else src.ctypes.data,
                       None if dst is None else dst.ctypes.data, int(key),
                       None if support_out is None else support_out.ctypes.data)
        t = ctypes.c_int64()
        _check(_lib.tc_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "tc_server_submit")
        self._keep[t.value] = (src, dst, support_out)
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """dict of the result, or None if not done (wait=False). A failed
        request gives status != 0 and the library's message in "error"."""
        r = _Result()
        st = _lib.tc_server_poll(self._h, int(ticket), 1 if wait else 0, ctypes.byref(r))
        if st == TC_EBUSY:
            return None
        _check(st, "tc_server_poll")
        src, dst, sup = self._keep.pop(int(ticket), (None, None, None))
        out = {"status": r.status, "cache_hit": bool(r.cache_hit), "count": r.count, "m": r.m,
               "t_submit": r.t_submit, "t_admit": r.t_admit, "t_ready": r.t_ready, "t_done": r.t_done}
        if r.status != TC_OK:
            out["error"] = _lib.tc_last_error().decode(errors="replace")
        if sup is not None and r.status == TC_OK:
            out["support"] = sup[:r.m]
        return out

    def cancel(self, ticket: int) -> bool:
        """True if the request was cancelled (or had already finished)."""
        st = _lib.tc_server_cancel(self._h, int(ticket))
        if st == TC_EBUSY:
            return False
        _check(st, "tc_server_cancel")
        return True

    def stats(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(2048)
        _check(_lib.tc_server_stats(self._h, buf, len(buf)), "tc_server_stats")
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            _lib.tc_server_destroy(self._h)
            self._h = ctypes.c_void_p(None)
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tc_graph_free(g: Graph):
    g.free()


class _ClassStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "workgroups", "rows", "table_keys", "tasks", "probes", "table_slots")]


def tc_graph_class_stats(g: Graph) -> dict:
    """{class name: {workgroups, rows, table_keys, tasks, probes, table_slots}}."""
    arr = (_ClassStats * TC_NUM_CLASSES)()
    _check(_lib.tc_graph_class_stats(g.handle, ctypes.cast(arr, _P)), "tc_graph_class_stats")
    out = {}
    for c in range(TC_NUM_CLASSES):
        out[_lib.tc_class_name(c).decode()] = {n: int(getattr(arr[c], n)) for n, _ in _ClassStats._fields_}
    return out


class Timer:
    """Phase timer: HIP events around every library launch made by this thread
    while attached (use as a context manager)."""

    def __init__(self, capacity: int = 4096):
        h = ctypes.c_void_p()
        _check(_lib.tc_timer_create(int(capacity), ctypes.byref(h)), "tc_timer_create")
        self._h = h

    def attach(self):
        _check(_lib.tc_timer_attach(self._h), "tc_timer_attach")

    @staticmethod
    def detach():
        _check(_lib.tc_timer_attach(None), "tc_timer_attach")

    def __enter__(self):
        self.attach()
        return self

    def __exit__(self, *exc):
        self.detach()

    def summary(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(1 << 20)
        _check(_lib.tc_timer_summary(self._h, buf, len(buf)), "tc_timer_summary")
        return json.loads(buf.value.decode())

    def reset(self):
        _check(_lib.tc_timer_reset(self._h), "tc_timer_reset")

    def free(self):
        if self._h:
            _lib.tc_timer_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
