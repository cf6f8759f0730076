"""Graphs stored renumbered by degree (GSM_GRAPH_DEGREE_ORDER) against the
oracle, through the C ABI.

Every result must be in the caller's ids: rows and counts equal the oracle's
on random instances (vertex and edge labels, induced, look-ahead, packed
frontier, every output path, sorted rows); candidate masks equal
oracle_filter's; root slices select the same roots, so the oracle's slice
counts of the 2^21-vertex, batching and serving workloads hold unchanged; in
the unique-subgraph mode the rows are exactly the oracle's embeddings that
satisfy the ordering constraints in the internal order, which the test
computes itself (ascending degree, ties by id).  Tolerance zero (integer
work).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

from golden.make_slice_counts import BATCH_SLICE, LARGE_MOD, SERVING_ARRIVALS, SERVING_MOD, fingerprint
from golden_io import GOLDEN

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def internal_id(g):
    """Internal number of each caller id: ascending degree, ties by id."""
    deg = np.diff(np.asarray(g.row_ptr, np.int64))
    orig = np.argsort(deg, kind="stable")
    new = np.empty(g.n, np.int64)
    new[orig] = np.arange(g.n)
    return new


def with_qlabels(qr, el):
    return W.Query(qr.q, qr.edges, qr.labels, None, -1.0, qr.name, np.asarray(el, np.int32))


def gpu_sorted(G, Q, **kw):
    c, _, _ = gsm.match(G, Q, **kw)
    c2, rows, _ = gsm.match(G, Q, rows="host", rows_cap=max(c, 1), sort_rows=True, **kw)
    assert c2 == c
    return c, rows


@pytest.mark.parametrize("seed", range(48))
def test_random_instances_degree_order(seed):
    rng = np.random.default_rng(141_000 + seed)
    n = int(rng.integers(2, 44))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.1, 0.6)), L, seed)
    qr = W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0, 0.6)), L, seed + 3)
    if seed % 4 == 3:  # edge labels
        EL = int(rng.integers(1, 4))
        g = W.with_edge_labels(g, EL, seed + 5)
        qr = with_qlabels(qr, rng.integers(0, EL, qr.ne))
    G = gsm.Graph.from_workload(g, validate=True, degree_order=True)
    Q = gsm.Query.from_workload(qr)
    induced = seed % 5 == 1
    kw = {} if oracle.match(g, qr, rows=False, induced=induced)[0] <= 1_000_000 else {"root": (0, 16, seed % 16)}
    c, r = oracle.match(g, qr, induced=induced, **kw)
    cg, rg = gpu_sorted(G, Q, induced=induced, lookahead=bool(seed % 2), filter_rounds=seed % 3,
                        pack_frontier=seed % 3 == 2, **kw)
    assert cg == c
    np.testing.assert_array_equal(rg, r)


def test_output_paths_degree_order():
    # device rows, host rows, host and device callbacks, sorted device rows,
    # and a truncated buffer: all in the caller's ids
    g = W.rmat_graph(10, 5, 0.57, 0.19, 0.19, 77)
    G = gsm.Graph.from_workload(g, validate=True, degree_order=True)
    for name in ("K3", "K4", "C4"):
        qr = W.shape(name)
        Q = gsm.Query.from_workload(qr)
        c, r = oracle.match(g, qr, threads=NCPU)
        print(name, c, flush=True)
        cg, rows, _ = gsm.match(G, Q, rows="host", rows_cap=c)
        assert cg == c
        np.testing.assert_array_equal(oracle.sort_rows(rows), r)
        dev = torch.full((c, qr.q), -1, dtype=torch.int32, device="cuda:0")
        cg, _, _ = gsm.match(G, Q, rows=dev)
        np.testing.assert_array_equal(oracle.sort_rows(dev.cpu().numpy()), r)
        cg, _, _ = gsm.match(G, Q, rows=dev, sort_rows=True)
        np.testing.assert_array_equal(dev.cpu().numpy(), r)
        got = []
        gsm.match(G, Q, emit=lambda a: got.append(np.array(a)), budget=gsm.min_budget(G, Q, host_rows=True) + (1 << 20))
        np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(got)), r)
        got = []

        def dsink(ptr, nrows, q):
            got.append(rows_from_device(ptr, nrows, q))
            return False

        gsm.match(G, Q, emit_device=dsink)
        np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(got)), r)
        if c > 3:
            small = torch.full((c // 2, qr.q), -1, dtype=torch.int32, device="cuda:0")
            cg, _, _ = gsm.match(G, Q, rows=small)  # truncated: the count stays exact
            assert cg == c
            part = small.cpu().numpy()
            assert (part >= 0).all() and (part < g.n).all()
            keys = {tuple(x) for x in r.tolist()}
            assert all(tuple(x) in keys for x in part.tolist())


def rows_from_device(ptr, nrows, q):
    """Copies a device chunk of rows to the host through the HIP runtime."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime already loaded (by soname)
    out = np.empty((nrows, q), np.int32)
    assert hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr), ctypes.c_size_t(out.nbytes),
                         2) == 0  # hipMemcpyDeviceToHost
    return out


@pytest.mark.parametrize("rounds", [0, 1, 3])
def test_filter_masks_degree_order(rounds):
    g = W.rmat_graph(12, 8, 0.57, 0.19, 0.19, 78)
    g = W.Graph(g.row_ptr, g.col, W.labels_zipf(g.n, 4, 1.0, 5), "labelled")
    G = gsm.Graph.from_workload(g, validate=True, degree_order=True)
    for k in range(4):
        qr = W.random_query(5, 0.4, 4, 900 + k)
        Q = gsm.Query.from_workload(qr)
        for root in (None, (1, 8, 3)):
            want = oracle.filter(g, qr, rounds=rounds, root=root)
            got = gsm.filter(G, Q, filter_rounds=rounds, root=root)
            np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("seed", range(30))
def test_unique_rows_in_internal_order(seed):
    rng = np.random.default_rng(142_000 + seed)
    n = int(rng.integers(3, 40))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.2, 0.8)), L, seed)
    qr = W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0.2, 1.0)), L, seed + 5)
    G = gsm.Graph.from_workload(g, validate=True, degree_order=True)
    Q = gsm.Query.from_workload(qr)
    aut, pairs = gsm.symmetry(Q)
    c, r = oracle.match(g, qr)
    cg, rg = gpu_sorted(G, Q, unique=True, lookahead=bool(seed % 2))
    assert cg * aut == c
    new = internal_id(g)
    keep = np.ones(r.shape[0], dtype=bool)
    for a, b in pairs:
        keep &= new[r[:, a]] < new[r[:, b]]
    np.testing.assert_array_equal(rg, r[keep])


def golden(fname):
    fp, rows = None, []
    for line in open(GOLDEN + "/" + fname):
        if line.startswith("# fingerprint"):
            fp = line.split()[2]
        elif not line.startswith("#") and line.strip():
            rows.append(line.split())
    return fp, rows


def test_large_graph_slices_degree_order():
    g = W.large_graph()
    fp, rows = golden("large_slice_counts.txt")
    shapes = []
    for r in rows:
        if r[0] not in shapes:
            shapes.append(r[0])
    assert fingerprint(g, [W.shape(s) for s in shapes]) == fp
    G = gsm.Graph.from_workload(g, degree_order=True)
    for name, rem, cnt in rows:
        Q = gsm.Query.from_workload(W.shape(name))
        print("large", name, "residue", rem, flush=True)
        c, _, _ = gsm.match(G, Q, root=(0, LARGE_MOD, int(rem)))
        assert c == int(cnt), (name, rem, c, cnt)
    # the unique triangle count is the textbook one whatever the numbering
    cu, _, _ = gsm.match(G, gsm.Query.from_workload(W.shape("K3")), unique=True)
    assert cu == oracle.triangles(g, threads=NCPU)


def test_batch_and_served_slices_degree_order():
    w = W.batch()
    fp, rows = golden("batch_slice_counts.txt")
    assert fingerprint(w.graph, w.queries) == fp
    expect = np.array([int(r[1]) for r in rows], dtype=np.uint64)
    G = gsm.Graph.from_workload(w.graph, degree_order=True)
    Qs = [gsm.Query.from_workload(q) for q in w.queries]
    print("batch of", len(Qs), flush=True)
    got = gsm.match_batch(G, Qs, root=BATCH_SLICE)
    np.testing.assert_array_equal(got, expect)
    del G
    w = W.serving(nq=SERVING_ARRIVALS)
    fp, rows = golden("serving_slice_counts.txt")
    assert fingerprint(w.graph, w.queries) == fp
    G = gsm.Graph.from_workload(w.graph, degree_order=True)
    pool = {}
    srv = gsm.Server(G, workers=4, arena_bytes=8 << 30, max_batch=32)
    try:
        tickets = []
        for k, qr in enumerate(w.queries):
            if id(qr) not in pool:
                pool[id(qr)] = gsm.Query.from_workload(qr)
            tickets.append(srv.submit(pool[id(qr)], root=(0, SERVING_MOD, k % SERVING_MOD)))
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    got = np.array([x["count"] for x in res], dtype=np.uint64)
    np.testing.assert_array_equal(got, np.array([int(r[2]) for r in rows], dtype=np.uint64))


def test_bad_ids_rejected_degree_order():
    # the renumbering range-checks offsets and ids even without validation
    rp = np.array([0, 1, 2], np.int64)
    with pytest.raises(gsm.GsmError) as e:
        gsm.Graph(rp, np.array([1, 5], np.int32), degree_order=True)
    assert e.value.status == 2  # GSM_E_BAD_GRAPH
    with pytest.raises(gsm.GsmError):
        gsm.Graph(np.array([0, 2, 1], np.int64), np.array([1, 0], np.int32), degree_order=True)
    G = gsm.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), degree_order=True)  # no vertices
    assert G.info()["n"] == 0


def test_device_pointers_and_strip_with_degree_order():
    # the renumbering also takes CSR arrays in device memory, and a cleaned
    # (stripped) adjacency; rows stay in the caller's ids
    g = W.rmat_graph(10, 5, 0.57, 0.19, 0.19, 91)
    g = W.Graph(g.row_ptr, g.col, W.labels_zipf(g.n, 3, 1.0, 4), "labelled")
    qr = W.random_query(4, 0.5, 3, 17)
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(g, qr)
    dev = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device="cuda:0")
    G = gsm.Graph(dev(g.row_ptr, torch.int64), dev(g.col, torch.int32), dev(g.labels, torch.int32),
                  degree_order=True)
    cg, rg = gpu_sorted(G, Q)
    assert cg == c
    np.testing.assert_array_equal(rg, r)
    # the same adjacency with every edge stored once and a self-loop added:
    # GSM_GRAPH_STRIP rebuilds it before the renumbering
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    keep = src < g.col
    half_src, half_dst = np.append(src[keep], 0), np.append(g.col[keep], 0)
    order = np.argsort(half_src, kind="stable")
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, half_src[order] + 1, 1)
    rp = np.cumsum(rp)
    G2 = gsm.Graph(rp, half_dst[order].astype(np.int32), g.labels, strip=True, degree_order=True)
    cg2, rg2 = gpu_sorted(G2, Q)
    assert cg2 == c
    np.testing.assert_array_equal(rg2, r)
