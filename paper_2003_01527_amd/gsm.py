"""Python binding of libgsm (include/gsm.h): argument marshalling only.

Every step of matching runs in the HIP library; this module converts numpy
arrays and torch tensors into the C ABI's pointers and sizes.  torch is used
for device buffers and streams when the caller passes device tensors.  If the
library is missing it is built; if it cannot be loaded, an error is raised:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libgsm.so")
_lib = None

MAXQ = 16
GRAPH_VALIDATE = 1
GRAPH_DEVICE_PTRS = 2
GRAPH_STRIP = 4
GRAPH_NO_HUB_BITMAPS = 8
GRAPH_DEGREE_ORDER = 16

STATUS = {0: "GSM_OK", 1: "GSM_E_INVALID_ARG", 2: "GSM_E_BAD_GRAPH", 3: "GSM_E_BAD_QUERY",
          4: "GSM_E_OOM", 5: "GSM_E_BUDGET", 6: "GSM_E_DEVICE", 7: "GSM_E_TRUNCATED",
          8: "GSM_E_CANCELLED", 9: "GSM_E_UNSUPPORTED", 10: "GSM_E_TIMEOUT"}


class GsmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("order", ctypes.c_int32 * MAXQ),
                ("parent", ctypes.c_int32 * MAXQ), ("backmask", ctypes.c_uint32 * MAXQ)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("q", ctypes.c_int32),
                ("candidates_root", ctypes.c_uint64), ("rows", ctypes.c_uint64 * MAXQ),
                ("pairs", ctypes.c_uint64 * MAXQ), ("chunks", ctypes.c_uint64 * MAXQ),
                ("probes", ctypes.c_uint64), ("alg_bytes", ctypes.c_uint64),
                ("filter_bytes", ctypes.c_uint64), ("expand_launches", ctypes.c_uint64),
                ("ms_expand", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("frontier_bytes", ctypes.c_uint64)]

    def as_dict(self):
        q = self.q
        return {"q": q, "candidates_root": self.candidates_root,
                "rows": list(self.rows[:q]), "pairs": list(self.pairs[:q]),
                "chunks": list(self.chunks[:q]), "probes": self.probes,
                "alg_bytes": self.alg_bytes, "filter_bytes": self.filter_bytes,
                "expand_launches": self.expand_launches, "ms_expand": self.ms_expand,
                "ms_total": self.ms_total, "frontier_bytes": self.frontier_bytes}


EMIT_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                           ctypes.c_uint64, ctypes.c_int32)


class MatchOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("memory_budget_bytes", ctypes.c_uint64),
                ("filter_rounds", ctypes.c_int32), ("use_degree", ctypes.c_int32),
                ("use_ne", ctypes.c_int32), ("rows_on_device", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p), ("root_qvertex", ctypes.c_int32),
                ("root_mod", ctypes.c_uint32), ("root_rem", ctypes.c_uint32),
                ("emit", EMIT_FN), ("emit_ctx", ctypes.c_void_p),
                ("stats", ctypes.POINTER(Stats)), ("tile_items", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("batch_heavy_pairs", ctypes.c_uint64),
                ("stage_bytes", ctypes.c_uint32)]


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # soname); loading it first makes libgsm bind to it, so device pointers
    # and streams from torch are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(_LIB_PATH):
        from . import _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    P = ctypes.POINTER
    lib.gsm_status_str.restype = ctypes.c_char_p
    lib.gsm_status_str.argtypes = [ctypes.c_int]
    lib.gsm_last_error.restype = ctypes.c_char_p
    lib.gsm_last_error.argtypes = []
    lib.gsm_graph_create.restype = ctypes.c_int
    lib.gsm_graph_create.argtypes = [i64, vp, vp, vp, u32, P(vp)]
    lib.gsm_graph_create_ex.argtypes = [i64, vp, vp, vp, vp, u32, P(vp)]
    lib.gsm_query_set_edge_labels.argtypes = [vp, vp]
    lib.gsm_testing_fail_allocations.argtypes = [i64]
    lib.gsm_testing_fail_allocations.restype = None
    lib.gsm_graph_destroy.argtypes = [vp]
    lib.gsm_graph_info.restype = ctypes.c_int
    lib.gsm_graph_info.argtypes = [vp, P(i64), P(i64), P(i32), P(i64)]
    lib.gsm_query_create.restype = ctypes.c_int
    lib.gsm_query_create.argtypes = [i32, i32, vp, vp, P(vp)]
    lib.gsm_query_destroy.argtypes = [vp]
    lib.gsm_query_plan.restype = ctypes.c_int
    lib.gsm_query_plan.argtypes = [vp, vp, P(PlanInfo)]
    lib.gsm_match_opts_init.argtypes = [P(MatchOpts)]
    lib.gsm_filter.restype = ctypes.c_int
    lib.gsm_filter.argtypes = [vp, vp, P(MatchOpts), vp]
    lib.gsm_match.restype = ctypes.c_int
    lib.gsm_match.argtypes = [vp, vp, P(MatchOpts), P(u64), vp, u64, P(u64)]
    lib.gsm_match_noalloc.restype = ctypes.c_int
    lib.gsm_match_noalloc.argtypes = [vp, vp, P(MatchOpts), P(u64), vp, u64, P(u64)]
    lib.gsm_match_min_budget.restype = ctypes.c_int
    lib.gsm_match_min_budget.argtypes = [vp, vp, i32, P(u64)]
    lib.gsm_sort_rows.argtypes = [vp, vp, u64, i32, i32, vp]
    lib.gsm_query_symmetry.argtypes = [vp, P(u64), vp, i32, P(i32)]
    lib.gsm_server_opts_init.argtypes = [P(ServerOpts)]
    lib.gsm_server_create.restype = ctypes.c_int
    lib.gsm_server_create.argtypes = [vp, P(ServerOpts), P(vp)]
    lib.gsm_server_submit.restype = ctypes.c_int
    lib.gsm_server_submit.argtypes = [vp, vp, P(u64)]
    lib.gsm_server_submit_slice.restype = ctypes.c_int
    lib.gsm_server_submit_slice.argtypes = [vp, vp, i32, u32, u32, P(u64)]
    lib.gsm_server_wait.restype = ctypes.c_int
    lib.gsm_server_wait.argtypes = [vp, u64, i32, P(Result)]
    lib.gsm_server_destroy.argtypes = [vp]
    lib.gsm_now_ns.restype = u64
    lib.gsm_now_ns.argtypes = []
    lib.gsm_match_batch.restype = ctypes.c_int
    lib.gsm_match_batch.argtypes = [vp, i32, P(vp), P(MatchOpts), P(u64)]
    _lib = lib
    return lib


def _check(st: int, allow=()):
    if st != 0 and st not in allow:
        raise GsmError(st, _load().gsm_last_error().decode())
    return st


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class Graph:
    """A data graph uploaded to the device (simple, undirected, sorted CSR)."""

    def __init__(self, row_ptr, col, labels=None, validate: bool = False, strip: bool = False,
                 edge_labels=None, hub_bitmaps: bool = True, degree_order: bool = False):
        lib = _load()
        flags = ((GRAPH_VALIDATE if validate else 0) | (GRAPH_STRIP if strip else 0)
                 | (0 if hub_bitmaps else GRAPH_NO_HUB_BITMAPS) | (GRAPH_DEGREE_ORDER if degree_order else 0))
        self._h = ctypes.c_void_p()
        if hasattr(row_ptr, "data_ptr"):  # torch tensors on the device
            flags |= GRAPH_DEVICE_PTRS
            n = int(row_ptr.shape[0]) - 1
            dp = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
            _check(lib.gsm_graph_create_ex(n, dp(row_ptr), dp(col), dp(labels), dp(edge_labels), flags,
                                           ctypes.byref(self._h)))
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            lb = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
            el = None if edge_labels is None else np.ascontiguousarray(edge_labels, dtype=np.int32)
            n = int(rp.shape[0]) - 1
            _check(lib.gsm_graph_create_ex(n, _p(rp), _p(cl), _p(lb), _p(el), flags, ctypes.byref(self._h)))
        self.n = n

    @classmethod
    def from_workload(cls, g, validate: bool = False, hub_bitmaps: bool = True, degree_order: bool = False):
        return cls(g.row_ptr, g.col, g.labels, validate, edge_labels=getattr(g, "edge_labels", None),
                   hub_bitmaps=hub_bitmaps, degree_order=degree_order)

    def info(self):
        n, nnz, ml, md = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(_load().gsm_graph_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(ml),
                                      ctypes.byref(md)))
        return {"n": n.value, "nnz": nnz.value, "max_label": ml.value, "max_degree": md.value}

    def close(self):
        if self._h:
            _load().gsm_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Query:
    """A connected query graph (1..16 vertices)."""

    def __init__(self, q: int, edges, labels=None, edge_labels=None):
        lib = _load()
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        lb = None if labels is None else np.ascontiguousarray(labels, dtype=np.int32)
        self._h = ctypes.c_void_p()
        _check(lib.gsm_query_create(int(q), int(e.shape[0]), _p(e), _p(lb), ctypes.byref(self._h)))
        self.q = int(q)
        if edge_labels is not None:
            el = np.ascontiguousarray(edge_labels, dtype=np.int32)
            _check(lib.gsm_query_set_edge_labels(self._h, _p(el)))

    @classmethod
    def from_workload(cls, qr):
        return cls(qr.q, qr.edges, qr.labels, getattr(qr, "edge_labels", None))

    def close(self):
        if self._h:
            _load().gsm_query_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FLAG_NO_OUTPUT_STAGING = 1
FLAG_SORT_ROWS = 2
FLAG_LOOKAHEAD = 4
FLAG_UNIQUE = 8
FLAG_INDUCED = 16
FLAG_PACK_FRONTIER = 32
FLAG_LOOKAHEAD2 = 64
FLAG_HOST_LEVELS = 128
FLAG_NO_GRAPH = 256


def make_opts(budget: int = 0, filter_rounds: int = 1, use_degree: bool = True, use_ne: bool = True,
              stream=None, root=None, tile_items: int = 0, wg_size: int = 0, profile: bool = False,
              stats: Optional[Stats] = None, stage_output: bool = True, sort_rows: bool = False,
              lookahead: bool = False, unique: bool = False, induced: bool = False, batch_heavy_pairs: int = 0,
              pack_frontier: bool = False, lookahead2: bool = False, host_levels: bool = False,
              no_graph: bool = False, stage_bytes: int = 0) -> MatchOpts:
    o = MatchOpts()
    _load().gsm_match_opts_init(ctypes.byref(o))
    o.memory_budget_bytes = int(budget)
    o.filter_rounds = int(filter_rounds)
    o.use_degree = 1 if use_degree else 0
    o.use_ne = 1 if use_ne else 0
    if stream is not None:
        o.hip_stream = ctypes.c_void_p(int(stream))
    if root is not None:
        o.root_qvertex, o.root_mod, o.root_rem = int(root[0]), int(root[1]), int(root[2])
    o.tile_items = int(tile_items)
    o.wg_size = int(wg_size)
    o.profile = 1 if profile else 0
    o.flags = ((0 if stage_output else FLAG_NO_OUTPUT_STAGING) | (FLAG_SORT_ROWS if sort_rows else 0)
               | (FLAG_LOOKAHEAD if lookahead else 0) | (FLAG_UNIQUE if unique else 0)
               | (FLAG_INDUCED if induced else 0) | (FLAG_PACK_FRONTIER if pack_frontier else 0)
               | (FLAG_LOOKAHEAD2 if lookahead2 else 0) | (FLAG_HOST_LEVELS if host_levels else 0)
               | (FLAG_NO_GRAPH if no_graph else 0))
    o.batch_heavy_pairs = int(batch_heavy_pairs)
    o.stage_bytes = int(stage_bytes)
    if stats is not None:
        stats.struct_size = ctypes.sizeof(Stats)
        o.stats = ctypes.pointer(stats)
    return o


def plan(graph: Graph, query: Query):
    info = PlanInfo()
    _check(_load().gsm_query_plan(graph._h, query._h, ctypes.byref(info)))
    q = info.q
    return list(info.order[:q]), list(info.parent[:q]), list(info.backmask[:q])


def filter(graph: Graph, query: Query, **kw) -> np.ndarray:
    out = np.zeros(graph.n, dtype=np.uint16)
    o = make_opts(**kw)
    _check(_load().gsm_filter(graph._h, query._h, ctypes.byref(o), _p(out)))
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # GSM_NOALLOC_SCRATCH_BYTES


def match(graph: Graph, query: Query, rows=None, rows_cap: Optional[int] = None, emit=None,
          emit_device=None, **kw):
    """Count (and list) embeddings.

    rows: None (count only), "host" (a numpy array of rows_cap rows), or a
    device torch int32 tensor of shape (cap, q).  emit: callable(rows ndarray)
    per output chunk (host rows).  emit_device: callable(device_ptr, nrows, q)
    per output chunk, rows left in device memory.  A callback returning a true
    value stops the match.  Returns (count, rows_or_None, stats dict).
    """
    return _match("gsm_match", graph, query, rows, rows_cap, emit, emit_device, **kw)


def match_noalloc(graph: Graph, query: Query, rows=None, rows_cap: Optional[int] = None, emit=None,
                  emit_device=None, **kw):
    """match() through gsm_match_noalloc: no device allocation inside the call."""
    return _match("gsm_match_noalloc", graph, query, rows, rows_cap, emit, emit_device, **kw)


def _match(entry: str, graph: Graph, query: Query, rows, rows_cap, emit, emit_device, **kw):
    lib = _load()
    st = Stats()
    o = make_opts(stats=st, **kw)
    cnt = ctypes.c_uint64(0)
    written = ctypes.c_uint64(0)
    out = None
    ptr, cap = None, 0
    keep = []
    if emit_device is not None:
        def _cbd(ctx, rp, nrows, q):
            return 1 if emit_device(ctypes.cast(rp, ctypes.c_void_p).value, int(nrows), int(q)) else 0
        cb = EMIT_FN(_cbd)
        keep.append(cb)
        o.emit = cb
        o.rows_on_device = 1
    elif emit is not None:
        def _cb(ctx, rp, nrows, q):
            a = np.ctypeslib.as_array(rp, shape=(int(nrows) * int(q),)).reshape(-1, int(q)).copy()
            return 1 if emit(a) else 0
        cb = EMIT_FN(_cb)
        keep.append(cb)
        o.emit = cb
    elif isinstance(rows, str) and rows == "host":
        if rows_cap is None:
            raise ValueError("rows_cap is required for host rows")
        out = np.zeros((int(rows_cap), query.q), dtype=np.int32)
        ptr, cap = _p(out), int(rows_cap)
    elif rows is not None:
        if not (hasattr(rows, "is_cuda") and rows.is_cuda):
            raise ValueError("rows must be 'host' or a device torch tensor")
        o.rows_on_device = 1
        out = rows
        ptr, cap = ctypes.c_void_p(rows.data_ptr()), int(rows.shape[0])
        if o.hip_stream is None:
            import torch
            o.hip_stream = ctypes.c_void_p(torch.cuda.current_stream(rows.device).cuda_stream)
    status = getattr(lib, entry)(graph._h, query._h, ctypes.byref(o), ctypes.byref(cnt), ptr, cap,
                                 ctypes.byref(written))
    _check(status, allow=(7,))
    count = int(cnt.value)
    if isinstance(out, np.ndarray):
        out = out[:int(written.value)]
    return count, out, st.as_dict()


class ServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("arena_bytes", ctypes.c_uint64),
                ("per_query_budget", ctypes.c_uint64), ("workers", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("tile_items", ctypes.c_int32),
                ("batch_heavy_pairs", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("count", ctypes.c_uint64), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("batch_size", ctypes.c_int32), ("worker", ctypes.c_int32),
                ("dev_start_ms", ctypes.c_double), ("dev_end_ms", ctypes.c_double)]


class Server:
    """Serving engine over a resident graph (gsm_server_*)."""

    def __init__(self, graph: Graph, arena_bytes: int = 0, per_query_budget: int = 0, workers: int = 0,
                 max_batch: int = 0, max_active: int = 0, wg_size: int = 0, tile_items: int = 0,
                 batch_heavy_pairs: int = 0):
        lib = _load()
        o = ServerOpts()
        lib.gsm_server_opts_init(ctypes.byref(o))
        o.arena_bytes, o.per_query_budget = int(arena_bytes), int(per_query_budget)
        o.workers, o.max_batch, o.max_active = int(workers), int(max_batch), int(max_active)
        o.wg_size, o.tile_items, o.batch_heavy_pairs = int(wg_size), int(tile_items), int(batch_heavy_pairs)
        self._graph = graph  # keeps the graph alive while the server runs
        self._h = ctypes.c_void_p()
        _check(lib.gsm_server_create(graph._h, ctypes.byref(o), ctypes.byref(self._h)))

    def submit(self, query: Query, root=None) -> int:
        """root: (query vertex, mod, rem) slice, or None for the whole query."""
        t = ctypes.c_uint64()
        if root is None:
            _check(_load().gsm_server_submit(self._h, query._h, ctypes.byref(t)))
        else:
            _check(_load().gsm_server_submit_slice(self._h, query._h, int(root[0]), int(root[1]), int(root[2]),
                                                   ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        r = Result()
        _check(_load().gsm_server_wait(self._h, ticket, timeout_ms, ctypes.byref(r)))
        return {"count": int(r.count), "t_submit_ns": int(r.t_submit_ns), "t_admit_ns": int(r.t_admit_ns),
                "t_done_ns": int(r.t_done_ns), "batch_size": int(r.batch_size), "worker": int(r.worker),
                "dev_start_ms": float(r.dev_start_ms), "dev_end_ms": float(r.dev_end_ms)}

    def close(self):
        if self._h:
            _load().gsm_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def testing_fail_allocations(after: int) -> None:
    """Test hook: after `after` more device allocations the library's
    allocations fail with GSM_E_OOM; after < 0 lifts the limit."""
    _load().gsm_testing_fail_allocations(int(after))


def now_ns() -> int:
    return int(_load().gsm_now_ns())


def symmetry(query: Query):
    """(|Aut(Q)|, [(a, b), ...]) with constraints f(a) < f(b) of the unique mode."""
    lib = _load()
    aut, n = ctypes.c_uint64(0), ctypes.c_int32(0)
    buf = np.zeros(2 * 16 * 16, dtype=np.int32)
    _check(lib.gsm_query_symmetry(query._h, ctypes.byref(aut), _p(buf), 16 * 16, ctypes.byref(n)))
    return int(aut.value), [(int(buf[2 * k]), int(buf[2 * k + 1])) for k in range(n.value)]


def sort_rows(graph: Graph, rows, stream=None):
    """Sorts rows (a numpy int32 (N, q) array, or a device torch int32 tensor
    of that shape) lexicographically in place on the device."""
    lib = _load()
    if isinstance(rows, np.ndarray):
        if rows.dtype != np.int32 or rows.ndim != 2 or not rows.flags["C_CONTIGUOUS"]:
            raise ValueError("rows must be a C-contiguous int32 (N, q) array")
        ptr, on_dev = _p(rows), 0
    else:
        if not (hasattr(rows, "is_cuda") and rows.is_cuda) or rows.dim() != 2 or not rows.is_contiguous():
            raise ValueError("rows must be a contiguous device (N, q) tensor")
        import torch
        if rows.dtype != torch.int32:
            raise ValueError("rows must be int32")
        ptr, on_dev = ctypes.c_void_p(rows.data_ptr()), 1
        if stream is None:
            stream = torch.cuda.current_stream(rows.device).cuda_stream
    st = ctypes.c_void_p(int(stream)) if stream is not None else None
    _check(lib.gsm_sort_rows(graph._h, ptr, int(rows.shape[0]), int(rows.shape[1]), on_dev, st))
    return rows


def min_budget(graph: Graph, query: Query, host_rows: bool = False) -> int:
    b = ctypes.c_uint64(0)
    _check(_load().gsm_match_min_budget(graph._h, query._h, 1 if host_rows else 0, ctypes.byref(b)))
    return int(b.value)


def match_batch(graph: Graph, queries: Sequence[Query], stats: Optional[Stats] = None, **kw) -> np.ndarray:
    counts = np.zeros(len(queries), dtype=np.uint64)
    arr = (ctypes.c_void_p * max(1, len(queries)))(*[q._h for q in queries])
    o = make_opts(stats=stats, **kw)
    _check(_load().gsm_match_batch(graph._h, len(queries), arr, ctypes.byref(o),
                                   counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return counts
