"""Seeded synthetic workloads: data graphs, query sets and arrival streams.

Both the CPU oracle and the HIP matcher read these inputs; this module holds
none of the matching arithmetic.  Generation runs in ``gen.c`` (compiled here
with gcc into ``libgsmgen.so``); this file marshals arguments and names the five
workloads used for parity tests and measurement:

* ``small``     Erdos-Renyi, 1,000 vertices, 4,000 edges, 4 uniform labels;
                10 four-vertex queries (3 paw, 3 path, 2 cycle, 2 star) found
                by random walk.
* ``powerlaw``  R-MAT (0.57, 0.19, 0.19), 2^17 vertices, edge factor 8,
                16 Zipf(1.0) labels; 20 induced random-walk queries with 5-6
                vertices and 5-9 edges.
* ``large``     R-MAT, 2^21 vertices, edge factor 16, unlabelled; queries
                triangle, 4-clique, 5-cycle and house+tail.
* ``batch``     the ``powerlaw`` graph; 512 induced random-walk queries, 3-8
                vertices, edge density in [0.3, 1.0].
* ``serving``   R-MAT, 2^20 vertices, edge factor 12, 32 Zipf(1.0) labels;
                10,000 induced random-walk queries, 3-8 vertices, with Poisson
                arrival times.

Random-walk queries follow the label-scalability protocol the paper adopts
(Sec. 4, query graphs made by random walks over a power-law-labelled data
graph).  Queries whose spanning-tree homomorphism bound exceeds ``2**32`` are
rejected so that every workload stays countable in 64 bits.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgsmgen.so")
_lib = None

SHAPE_INDUCED, SHAPE_PAW, SHAPE_P4, SHAPE_C4, SHAPE_STAR = 0, 1, 2, 3, 4
CAP_DEFAULT = float(2 ** 32)


def build(force: bool = True) -> str:
    """Compile gen.c into libgsmgen.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", _SRC, "-o", tmp,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    i64, i32, u64, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    lib.gen_free.argtypes = [vp]
    lib.gen_substream_seed.restype = u64
    lib.gen_substream_seed.argtypes = [u64, u64]
    lib.gen_er_csr.restype = i64
    lib.gen_er_csr.argtypes = [i64, i64, u64, P(vp), P(vp)]
    lib.gen_rmat_csr.restype = i64
    lib.gen_rmat_csr.argtypes = [ctypes.c_int, dbl, dbl, dbl, dbl, u64, P(vp), P(vp)]
    lib.gen_labels_uniform.argtypes = [i64, i32, u64, vp]
    lib.gen_labels_zipf.argtypes = [i64, i32, dbl, u64, vp]
    lib.gen_query_set.restype = i64
    lib.gen_query_set.argtypes = [i64, vp, vp, vp, i32, i32, i32, i32, i32, dbl, dbl, dbl, u64, i32,
                                  i64, i32, vp, vp, vp, vp, vp, vp]
    lib.gen_tree_hom_bound.restype = dbl
    lib.gen_tree_hom_bound.argtypes = [i64, vp, vp, vp, i32, i32, vp, vp]
    lib.gen_poisson_arrivals.argtypes = [i64, dbl, u64, vp]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def substream(master: int, k: int) -> int:
    return int(_load().gen_substream_seed(master, k))


@dataclass
class Graph:
    """Simple undirected graph in CSR with sorted rows (int64 offsets, int32 ids)."""
    row_ptr: np.ndarray
    col: np.ndarray
    labels: Optional[np.ndarray] = None  # int32 per vertex, None = unlabelled
    name: str = ""
    edge_labels: Optional[np.ndarray] = None  # int32 per CSR entry (both directions alike), None = none

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


@dataclass
class Query:
    """Connected query graph: q vertices, undirected edge list, optional labels."""
    q: int
    edges: np.ndarray                    # int32 (ne, 2)
    labels: Optional[np.ndarray] = None  # int32 (q,)
    source: Optional[np.ndarray] = None  # data vertices the query was drawn from
    bound: float = -1.0                  # spanning-tree homomorphism bound
    name: str = ""
    edge_labels: Optional[np.ndarray] = None  # int32 (ne,) per edge, None = unconstrained

    @property
    def ne(self) -> int:
        return int(self.edges.shape[0])


@dataclass
class Workload:
    name: str
    graph: Graph
    queries: List[Query] = field(default_factory=list)
    arrivals: Optional[np.ndarray] = None
    candidates_examined: int = 0


def _take_csr(n: int, nnz: int, rp_p: ctypes.c_void_p, col_p: ctypes.c_void_p):
    lib = _load()
    rp = np.ctypeslib.as_array(ctypes.cast(rp_p, ctypes.POINTER(ctypes.c_int64)), shape=(n + 1,)).copy()
    if nnz > 0:
        col = np.ctypeslib.as_array(ctypes.cast(col_p, ctypes.POINTER(ctypes.c_int32)), shape=(nnz,)).copy()
    else:
        col = np.zeros(0, dtype=np.int32)
    lib.gen_free(rp_p)
    lib.gen_free(col_p)
    return rp, col


def er_graph(n: int, m: int, seed: int) -> Graph:
    rp_p, col_p = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = _load().gen_er_csr(n, m, seed, ctypes.byref(rp_p), ctypes.byref(col_p))
    if nnz < 0:
        raise ValueError("gen_er_csr failed")
    rp, col = _take_csr(n, nnz, rp_p, col_p)
    return Graph(rp, col)


def rmat_graph(scale: int, ef: float, a: float, b: float, c: float, seed: int) -> Graph:
    rp_p, col_p = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = _load().gen_rmat_csr(scale, ef, a, b, c, seed, ctypes.byref(rp_p), ctypes.byref(col_p))
    if nnz < 0:
        raise ValueError("gen_rmat_csr failed")
    rp, col = _take_csr(1 << scale, nnz, rp_p, col_p)
    return Graph(rp, col)


def labels_uniform(n: int, L: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().gen_labels_uniform(n, L, seed, _ptr(out))
    return out


def labels_zipf(n: int, L: int, s: float, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().gen_labels_zipf(n, L, s, seed, _ptr(out))
    return out


def query_set(g: Graph, want: int, seed: int, kind: int = SHAPE_INDUCED, k_min: int = 3,
              k_max: int = 8, e_min: int = 0, e_max: int = 120, dens_min: float = 0.0,
              dens_max: float = 1.0, cap: float = CAP_DEFAULT, max_candidates: int = 0,
              nthreads: Optional[int] = None) -> tuple:
    """Accepted random-walk queries, in candidate order; also returns #candidates examined."""
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    if max_candidates <= 0:
        max_candidates = 200 * want + 20_000
    q = np.zeros(want, np.int32)
    ne = np.zeros(want, np.int32)
    edges = np.zeros((want, 240), np.int32)
    labels = np.zeros((want, 16), np.int32)
    source = np.zeros((want, 16), np.int32)
    bound = np.zeros(want, np.float64)
    lab = g.labels
    examined = _load().gen_query_set(g.n, _ptr(g.row_ptr), _ptr(g.col), _ptr(lab), kind, k_min, k_max,
                                     e_min, e_max, dens_min, dens_max, cap, seed, want, max_candidates,
                                     nthreads, _ptr(q), _ptr(ne), _ptr(edges), _ptr(labels),
                                     _ptr(source), _ptr(bound))
    if examined < 0:
        raise RuntimeError("query generator: too few accepted candidates")
    out = []
    for j in range(want):
        qq, m = int(q[j]), int(ne[j])
        out.append(Query(qq, edges[j, :2 * m].reshape(m, 2).copy(),
                         labels[j, :qq].copy() if lab is not None else None,
                         source[j, :qq].copy(), float(bound[j])))
    return out, int(examined)


def tree_hom_bound(g: Graph, qr: Query) -> float:
    e = np.ascontiguousarray(qr.edges, dtype=np.int32)
    ql = None if qr.labels is None else np.ascontiguousarray(qr.labels, dtype=np.int32)
    return float(_load().gen_tree_hom_bound(g.n, _ptr(g.row_ptr), _ptr(g.col), _ptr(g.labels), qr.q,
                                            qr.ne, _ptr(e), _ptr(ql)))


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().gen_poisson_arrivals(count, rate, seed, _ptr(out))
    return out


# ------------------------------------------------------------- shapes --

def shape(name: str) -> Query:
    """Named unlabelled query shapes."""
    E = {
        "K2": [(0, 1)],
        "K3": [(0, 1), (1, 2), (0, 2)],
        "K4": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
        "C4": [(0, 1), (1, 2), (2, 3), (0, 3)],
        "C5": [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4)],
        "P3": [(0, 1), (1, 2)],
        "P4": [(0, 1), (1, 2), (2, 3)],
        "paw": [(0, 1), (1, 2), (0, 2), (0, 3)],
        "star3": [(0, 1), (0, 2), (0, 3)],
        # square 0-1-2-3-0, roof vertex 4 on 0 and 1, tail vertex 5 on 4
        "house_tail": [(0, 1), (1, 2), (2, 3), (0, 3), (0, 4), (1, 4), (4, 5)],
    }[name]
    q = 1 + max(max(e) for e in E)
    return Query(q, np.array(E, dtype=np.int32), None, None, -1.0, name)


# ---------------------------------------------------------- workloads --

def small(seed: int = 1) -> Workload:
    g = er_graph(1000, 4000, substream(seed, 0))
    g.labels = labels_uniform(g.n, 4, substream(seed, 1))
    g.name = "er_n1000_m4000_L4"
    queries = []
    examined = 0
    for k, (kind, cnt) in enumerate([(SHAPE_PAW, 3), (SHAPE_P4, 3), (SHAPE_C4, 2), (SHAPE_STAR, 2)]):
        qs, ex = query_set(g, cnt, substream(seed, 2 + k), kind=kind, k_min=4, k_max=4, cap=0.0)
        for qr in qs:
            qr.name = {SHAPE_PAW: "paw", SHAPE_P4: "P4", SHAPE_C4: "C4", SHAPE_STAR: "star3"}[kind]
        queries += qs
        examined += ex
    return Workload("small", g, queries, None, examined)


def powerlaw_graph(seed: int = 2) -> Graph:
    g = rmat_graph(17, 8.0, 0.57, 0.19, 0.19, substream(seed, 0))
    g.labels = labels_zipf(g.n, 16, 1.0, substream(seed, 1))
    g.name = "rmat_s17_ef8_L16zipf1"
    return g


def powerlaw(seed: int = 2, nq: int = 20) -> Workload:
    g = powerlaw_graph(seed)
    qs, ex = query_set(g, nq, substream(seed, 2), k_min=5, k_max=6, e_min=5, e_max=9)
    for i, qr in enumerate(qs):
        qr.name = "pl%02d" % i
    return Workload("powerlaw", g, qs, None, ex)


def large_graph(seed: int = 3) -> Graph:
    g = rmat_graph(21, 16.0, 0.57, 0.19, 0.19, substream(seed, 0))
    g.name = "rmat_s21_ef16_unlabelled"
    return g


def large(seed: int = 3) -> Workload:
    g = large_graph(seed)
    return Workload("large", g, [shape("K3"), shape("K4"), shape("C5"), shape("house_tail")])


def batch(seed: int = 4, nq: int = 512, graph_seed: int = 2, cap: float = CAP_DEFAULT) -> Workload:
    """cap: spanning-tree bound above which a query is rejected (2^32 by
    default; a small cap such as 2^20 gives a mix of light queries)."""
    g = powerlaw_graph(graph_seed)
    qs, ex = query_set(g, nq, substream(seed, 2), k_min=3, k_max=8, dens_min=0.3, dens_max=1.0, cap=cap)
    for i, qr in enumerate(qs):
        qr.name = "b%03d" % i
    return Workload("batch", g, qs, None, ex)


def serving_graph(seed: int = 5) -> Graph:
    g = rmat_graph(20, 12.0, 0.57, 0.19, 0.19, substream(seed, 0))
    g.labels = labels_zipf(g.n, 32, 1.0, substream(seed, 1))
    g.name = "rmat_s20_ef12_L32zipf1"
    return g


def serving(seed: int = 5, nq: int = 10_000, rate: float = 1000.0, pool: int = 1000) -> Workload:
    """Arrivals draw (uniformly, seeded) from a pool of `pool` distinct accepted queries:
    the spanning-tree bound costs ~0.1 s of CPU per candidate on this graph, so
    drawing 10,000 distinct ones would dominate set-up time.  Every arrival is
    matched from scratch; nothing is cached between arrivals."""
    g = serving_graph(seed)
    qs, ex = query_set(g, min(pool, nq), substream(seed, 2), k_min=3, k_max=8)
    for i, qr in enumerate(qs):
        qr.name = "s%04d" % i
    pick = np.empty(nq, dtype=np.int32)
    _load().gen_labels_uniform(nq, len(qs), substream(seed, 4), _ptr(pick))
    arr = poisson_arrivals(nq, rate, substream(seed, 3))
    w = Workload("serving", g, [qs[int(i)] for i in pick], arr, ex)
    return w


# ------------------------------------------------ tiny random instances --

def from_edges(n: int, edges, labels=None, name: str = "") -> Graph:
    """CSR of a simple undirected graph given as an edge list (duplicates and
    self-loops removed)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]]) if e.shape[0] else np.zeros((0, 2), np.int64)
    key = np.unique(both[:, 0] * n + both[:, 1]) if both.shape[0] else np.zeros(0, np.int64)
    src, dst = key // n, key % n
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    lab = None if labels is None else np.asarray(labels, dtype=np.int32)
    return Graph(rp, dst.astype(np.int32), lab, name)


def with_edge_labels(g: Graph, L: int, seed: int) -> Graph:
    """A copy of g whose undirected edges carry uniform labels in [0, L)
    (numpy PCG64 seeded); both CSR entries of an edge get its label."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    key = np.minimum(src, dst) * max(n, 1) + np.maximum(src, dst)
    uniq, inv = np.unique(key, return_inverse=True)
    lab = np.random.default_rng(seed).integers(0, max(L, 1), uniq.shape[0]).astype(np.int32)
    return Graph(g.row_ptr, g.col, g.labels, g.name, lab[inv])


def random_graph(n: int, p: float, L: int, seed: int) -> Graph:
    """G(n, p) with L uniform labels (L = 0: unlabelled), numpy PCG64 seeded."""
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p
    lab = None if L <= 0 else rng.integers(0, L, n).astype(np.int32)
    return from_edges(n, np.stack([iu[0][keep], iu[1][keep]], 1), lab)


def random_query(q: int, p: float, L: int, seed: int) -> Query:
    """Connected query: a random spanning tree plus each other pair with prob. p."""
    rng = np.random.default_rng(seed)
    E = set()
    perm = rng.permutation(q)
    for i in range(1, q):
        a, b = int(perm[i]), int(perm[rng.integers(0, i)])
        E.add((min(a, b), max(a, b)))
    for a in range(q):
        for b in range(a + 1, q):
            if rng.random() < p:
                E.add((a, b))
    edges = np.array(sorted(E), dtype=np.int32).reshape(-1, 2)
    lab = None if L <= 0 else rng.integers(0, L, q).astype(np.int32)
    return Query(q, edges, lab)
