"""HIP path vs the CPU oracle, element by element, through the C ABI.

Counts are compared exactly; row sets are compared after sorting (the GPU's
row order depends on atomics).  Filter masks are compared bit for bit.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def gpu_rows(G, Q, **kw):
    cnt, _, _ = gsm.match(G, Q, **kw)
    c2, rows, _ = gsm.match(G, Q, rows="host", rows_cap=max(cnt, 1), **kw)
    assert c2 == cnt
    return cnt, oracle.sort_rows(rows)


@pytest.fixture(scope="module")
def small():
    w = W.small()
    return w, gsm.Graph.from_workload(w.graph, validate=True)


@pytest.fixture(scope="module")
def powerlaw():
    w = W.powerlaw()
    return w, gsm.Graph.from_workload(w.graph)


def test_small_workload_rows(small):
    w, G = small
    for qr in w.queries:
        print("small", qr.name, flush=True)
        Q = gsm.Query.from_workload(qr)
        c, r = oracle.match(w.graph, qr)
        cg, rg = gpu_rows(G, Q)
        assert cg == c, qr.name
        np.testing.assert_array_equal(rg, r)


@pytest.mark.parametrize("seed", range(120))
def test_random_instances(seed):
    rng = np.random.default_rng(40_000 + seed)
    n = int(rng.integers(2, 48))
    L = int(rng.integers(0, 4))
    g = W.random_graph(n, float(rng.uniform(0.05, 0.6)), L, seed)
    qr = W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0, 0.5)), L, seed + 7)
    G = gsm.Graph.from_workload(g, validate=True)
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(g, qr)
    rounds = seed % 4
    cg, rg = gpu_rows(G, Q, filter_rounds=rounds, use_ne=bool(seed % 2))
    assert cg == c
    np.testing.assert_array_equal(rg, r)


@pytest.mark.parametrize("rounds", [0, 1, 3])
@pytest.mark.parametrize("use_deg,use_ne", [(False, False), (True, False), (True, True)])
def test_filter_bits_powerlaw(powerlaw, rounds, use_deg, use_ne):
    w, G = powerlaw
    for qr in w.queries[:6]:
        Q = gsm.Query.from_workload(qr)
        a = oracle.filter(w.graph, qr, rounds=rounds, use_deg=use_deg, use_ne=use_ne)
        b = gsm.filter(G, Q, filter_rounds=rounds, use_degree=use_deg, use_ne=use_ne)
        np.testing.assert_array_equal(a, b)


def test_filter_bits_with_root_slice(powerlaw):
    w, G = powerlaw
    qr = w.queries[3]
    Q = gsm.Query.from_workload(qr)
    for root in [(0, 7, 3), (qr.q - 1, 64, 0)]:
        a = oracle.filter(w.graph, qr, rounds=2, root=root)
        b = gsm.filter(G, Q, filter_rounds=2, root=root)
        np.testing.assert_array_equal(a, b)


def test_plan_matches_oracle(powerlaw, small):
    for w, G in (powerlaw, small):
        for qr in w.queries:
            Q = gsm.Query.from_workload(qr)
            expect = oracle.plan(qr.q, qr.edges, qr.labels, w.graph.labels, w.graph.degrees())
            assert tuple(gsm.plan(G, Q)) == tuple(expect)


@pytest.mark.parametrize("k", range(20))
def test_powerlaw_root_slice_counts(powerlaw, k):
    w, G = powerlaw
    qr = w.queries[k]
    Q = gsm.Query.from_workload(qr)
    root = (k % qr.q, 64, k % 5)
    print("powerlaw slice", qr.name, root, flush=True)
    c, _ = oracle.match(w.graph, qr, rows=False, threads=NCPU, root=root)
    cg, _, _ = gsm.match(G, Q, root=root)
    assert cg == c


@pytest.mark.parametrize("k", [9, 10, 13])
def test_powerlaw_full_counts(powerlaw, k):
    w, G = powerlaw
    qr = w.queries[k]
    c, _ = oracle.match(w.graph, qr, rows=False, threads=NCPU)
    cg, _, st = gsm.match(G, gsm.Query.from_workload(qr))
    assert cg == c
    assert st["rows"][qr.q - 1] == c


def test_powerlaw_slice_rows_and_tiny_budgets(powerlaw):
    """Sorted rows on a slice, identical across budgets down to a few rows per chunk."""
    w, G = powerlaw
    qr = w.queries[9]
    Q = gsm.Query.from_workload(qr)
    root = (0, 128, 1)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root)
    assert 0 < c < 5_000_000
    lo = gsm.min_budget(G, Q, host_rows=True)
    for budget in (0, lo + (1 << 20), lo + (1 << 16)):
        cg, rg = gpu_rows(G, Q, root=root, budget=budget)
        assert cg == c, budget
        np.testing.assert_array_equal(rg, r)


@pytest.mark.parametrize("wg,items", [(128, 1), (256, 2), (256, 4), (512, 8)])
def test_launch_shapes_agree(small, wg, items):
    w, G = small
    for qr in w.queries[:4]:
        Q = gsm.Query.from_workload(qr)
        c, r = oracle.match(w.graph, qr)
        cg, rg = gpu_rows(G, Q, wg_size=wg, tile_items=items)
        assert cg == c
        np.testing.assert_array_equal(rg, r)


def test_device_rows_truncation_and_emit(small):
    import torch
    w, G = small
    qr = w.queries[3]  # a path query with thousands of embeddings
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(w.graph, qr)
    dev = torch.full((c, qr.q), -1, dtype=torch.int32, device="cuda")
    cg, out, _ = gsm.match(G, Q, rows=dev)
    torch.cuda.synchronize()
    assert cg == c
    np.testing.assert_array_equal(oracle.sort_rows(out.cpu().numpy()), r)
    # truncated: count exact, every written row is an embedding
    small_dev = torch.full((c // 3, qr.q), -1, dtype=torch.int32, device="cuda")
    cg, out, _ = gsm.match(G, Q, rows=small_dev)
    torch.cuda.synchronize()
    assert cg == c
    got = out.cpu().numpy()
    rset = set(map(tuple, r.tolist()))
    assert all(tuple(x) in rset for x in got.tolist())
    # host truncation
    cg, got, _ = gsm.match(G, Q, rows="host", rows_cap=10)
    assert cg == c and got.shape == (10, qr.q)
    assert all(tuple(x) in rset for x in got.tolist())
    # host emit callback, chunked by a small budget
    chunks = []
    lo = gsm.min_budget(G, Q, host_rows=True)
    cg, _, st = gsm.match(G, Q, emit=lambda a: chunks.append(a) and False, budget=lo + 20_000)
    assert cg == c
    np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(chunks)), r)
    # device emit callback sees every row once
    seen = []

    def sink(ptr, nrows, q):
        buf = torch.empty((nrows, q), dtype=torch.int32)
        import ctypes
        lib = ctypes.CDLL("libamdhip64.so.7")  # the runtime already loaded (by soname)
        lib.hipMemcpy(ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(ptr),
                      ctypes.c_size_t(nrows * q * 4), 2)
        seen.append(buf.numpy().copy())
        return False
    cg, _, _ = gsm.match(G, Q, emit_device=sink, budget=lo + 20_000)
    assert cg == c
    np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(seen)), r)


def test_single_vertex_and_edge_queries(small):
    w, G = small
    for qr in (W.Query(1, np.zeros((0, 2), np.int32), np.array([2], np.int32)),
               W.Query(2, np.array([[0, 1]], np.int32), np.array([1, 3], np.int32))):
        c, r = oracle.match(w.graph, qr)
        cg, rg = gpu_rows(G, gsm.Query.from_workload(qr))
        assert cg == c
        np.testing.assert_array_equal(rg, r)


def test_budget_error(small):
    w, G = small
    Q = gsm.Query.from_workload(w.queries[0])
    with pytest.raises(gsm.GsmError) as ei:
        gsm.match(G, Q, budget=1024)
    assert ei.value.status == 5
    lo = gsm.min_budget(G, Q)
    with pytest.raises(gsm.GsmError) as ei:
        gsm.match(G, Q, budget=lo - 100)
    assert ei.value.status == 5
    c, _ = oracle.match(w.graph, w.queries[0], rows=False)
    assert gsm.match(G, Q, budget=lo)[0] == c


def test_graph_validation_on_device_errors():
    # asymmetric
    with pytest.raises(gsm.GsmError) as ei:
        gsm.Graph(np.array([0, 1, 1]), np.array([1], np.int32), validate=True)
    assert ei.value.status == 2
    # unsorted row
    rp = np.array([0, 2, 3, 4])
    col = np.array([2, 1, 0, 0], np.int32)
    with pytest.raises(gsm.GsmError):
        gsm.Graph(rp, col, validate=True)


@pytest.mark.parametrize("extra", [1 << 12, 1 << 16, 1 << 22])
def test_device_sink_chunks(powerlaw, extra):
    """Rows handed to a device sink chunk by chunk are exactly the oracle's,
    for several chunk sizes; a sink that stops early cancels the match."""
    import ctypes
    import torch
    w, G = powerlaw
    qr = w.queries[9]
    root = (0, 32, 1)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root)
    Q = gsm.Query.from_workload(qr)
    lib = ctypes.CDLL("libamdhip64.so.7")
    seen = []

    def sink(ptr, nrows, q):
        buf = torch.empty((nrows, q), dtype=torch.int32)
        assert lib.hipMemcpy(ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(ptr),
                             ctypes.c_size_t(nrows * q * 4), 2) == 0
        seen.append(buf.numpy().copy())
        return False
    budget = gsm.min_budget(G, Q, host_rows=True) + extra
    cg, _, st = gsm.match(G, Q, emit_device=sink, root=root, budget=budget)
    assert cg == c
    np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(seen)), r)
    calls = []

    def stop(ptr, nrows, q):
        calls.append(nrows)
        return len(calls) >= 2
    try:
        gsm.match(G, Q, emit_device=stop, root=root, budget=budget)
        assert len(calls) < 2  # finished before a second chunk
    except gsm.GsmError as e:
        assert e.status == 8 and len(calls) == 2
