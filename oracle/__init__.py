"""CPU oracle for the subgraph matcher.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

* ``match``      all embeddings by depth-first backtracking (gsm_oracle.c)
* ``filter``     the filtering stage's candidate sets (gsm_oracle.c)
* ``triangles``  textbook forward triangle count, an independent pin (triangles.c)
* ``plan``       the host pre-computation's visiting order (plan.py)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .plan import plan  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "gsm_oracle.c"), os.path.join(_HERE, "triangles.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", *_SRCS, "-o", tmp,
                               "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
        lib.oracle_match.restype = ctypes.c_int
        lib.oracle_match.argtypes = [i64, vp, vp, vp, i32, i32, vp, vp, i32, u32, u32, i32, i32,
                                     ctypes.POINTER(u64), ctypes.POINTER(vp)]
        lib.oracle_match_ex.restype = ctypes.c_int
        lib.oracle_match_ex.argtypes = [i64, vp, vp, vp, i32, i32, vp, vp, i32, u32, u32, i32, i32, i32,
                                        ctypes.POINTER(u64), ctypes.POINTER(vp)]
        lib.oracle_filter.restype = ctypes.c_int
        lib.oracle_filter.argtypes = [i64, vp, vp, vp, i32, i32, vp, vp, i32, i32, i32, i32, u32, u32, vp]
        lib.oracle_triangles.restype = i64
        lib.oracle_triangles.argtypes = [i64, vp, vp, i32]
        lib.oracle_slice_hash.restype = u64
        lib.oracle_slice_hash.argtypes = [u64]
        lib.oracle_free.argtypes = [vp]
        lib.oracle_match_el.restype = ctypes.c_int
        lib.oracle_match_el.argtypes = [i64, vp, vp, vp, vp, i32, i32, vp, vp, vp, i32, u32, u32, i32, i32, i32,
                                        ctypes.POINTER(u64), ctypes.POINTER(vp)]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    lab = None if g.labels is None else np.ascontiguousarray(g.labels, dtype=np.int32)
    return rp, col, lab


def _edge_labels(x):
    el = getattr(x, "edge_labels", None)
    return None if el is None else np.ascontiguousarray(el, dtype=np.int32)


def _query_arrays(qr):
    e = np.ascontiguousarray(np.asarray(qr.edges, dtype=np.int32).reshape(-1, 2))
    ql = None if qr.labels is None else np.ascontiguousarray(qr.labels, dtype=np.int32)
    return e, ql


def sort_rows(rows: np.ndarray) -> np.ndarray:
    """Rows in lexicographic ascending order."""
    if rows.shape[0] == 0:
        return rows
    idx = np.lexsort(tuple(rows[:, j] for j in range(rows.shape[1] - 1, -1, -1)))
    return rows[idx]


def match(g, qr, rows=True, threads=1, root=None, induced=False):
    """(count, rows) of all embeddings of query qr in graph g.

    rows are int32 (count, q) in query-vertex-id columns, sorted ascending; None
    when rows=False.  root = (query_vertex, mod, rem) restricts to embeddings
    whose image of query_vertex lies in that slice of the slice hash.  induced:
    non-adjacent query vertices must map to non-adjacent data vertices too.
    Edge labels are taken from g.edge_labels (per CSR entry) and
    qr.edge_labels (per query edge) when present.
    """
    lib = _load()
    rp, col, lab = _graph_arrays(g)
    e, ql = _query_arrays(qr)
    rq, rm, rr = (-1, 0, 0) if root is None else root
    cnt = ctypes.c_uint64(0)
    out = ctypes.c_void_p()
    gel, qel = _edge_labels(g), _edge_labels(qr)
    rc = lib.oracle_match_el(g.n, _p(rp), _p(col), _p(lab), _p(gel), qr.q, e.shape[0], _p(e), _p(ql), _p(qel),
                             rq, rm, rr, 1 if rows else 0, threads, 1 if induced else 0, ctypes.byref(cnt),
                             ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("oracle_match failed (%d)" % rc)
    count = int(cnt.value)
    if not rows:
        return count, None
    if count:
        arr = np.ctypeslib.as_array(ctypes.cast(out, ctypes.POINTER(ctypes.c_int32)),
                                    shape=(count, qr.q)).copy()
    else:
        arr = np.zeros((0, qr.q), dtype=np.int32)
    lib.oracle_free(out)
    return count, sort_rows(arr)


def filter(g, qr, rounds=1, use_deg=True, use_ne=True, root=None):
    """uint16 per data vertex; bit u set when v is a candidate of query vertex u."""
    lib = _load()
    rp, col, lab = _graph_arrays(g)
    e, ql = _query_arrays(qr)
    rq, rm, rr = (-1, 0, 0) if root is None else root
    out = np.zeros(g.n, dtype=np.uint16)
    rc = lib.oracle_filter(g.n, _p(rp), _p(col), _p(lab), qr.q, e.shape[0], _p(e), _p(ql), rounds,
                           1 if use_deg else 0, 1 if use_ne else 0, rq, rm, rr, _p(out))
    if rc != 0:
        raise RuntimeError("oracle_filter failed (%d)" % rc)
    return out


def triangles(g, threads=1):
    """Number of triangles of g (each unordered triple once)."""
    rp, col, _ = _graph_arrays(g)
    r = _load().oracle_triangles(g.n, _p(rp), _p(col), threads)
    if r < 0:
        raise RuntimeError("oracle_triangles failed")
    return int(r)


def slice_hash(x: int) -> int:
    return int(_load().oracle_slice_hash(x))
