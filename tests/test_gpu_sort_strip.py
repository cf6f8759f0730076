"""Sorted output (the result as a sorted set of rows) and CSR stripping,
through the C ABI on the device.

Row order is checked against numpy's lexsort of the same rows, and the sorted
embedding lists against the oracle's sorted result set with no host-side
sorting of the GPU output.  Stripped graphs are checked against the CSR that
the workload module builds from the cleaned edge list.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu


def lex(rows):
    rows = np.asarray(rows)
    if rows.shape[0] == 0:
        return rows
    return rows[np.lexsort(rows.T[::-1])]


def edgeless(n):
    return gsm.Graph(np.zeros(n + 1, np.int64), np.zeros(0, np.int32))


@pytest.fixture(scope="module")
def graphs():
    # vertex counts whose id widths are 1, 10, 17 and 25 bits
    return {n: edgeless(n) for n in (2, 1000, 1 << 17, 1 << 25)}


@pytest.mark.parametrize("n", [2, 1000, 1 << 17, 1 << 25])
@pytest.mark.parametrize("q", [1, 2, 3, 5, 8, 16])
@pytest.mark.parametrize("N", [0, 1, 2, 2047, 2048, 2049, 70_001])
def test_sort_device_rows_random(graphs, n, q, N):
    print("sort", n, q, N, flush=True)
    rng = np.random.default_rng(n * 131 + q * 7 + N)
    # few distinct values in some columns, so equal prefixes and equal rows occur
    hi = np.where(rng.random(q) < 0.3, min(n, 3), n)
    rows = np.stack([rng.integers(0, h, N) for h in hi], 1).astype(np.int32).reshape(N, q)
    t = torch.from_numpy(rows.copy()).cuda()
    gsm.sort_rows(graphs[n], t)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(t.cpu().numpy(), lex(rows))


@pytest.mark.parametrize("N", [3, 5000])
def test_sort_host_rows(graphs, N):
    rng = np.random.default_rng(N)
    rows = rng.integers(0, 1000, (N, 4)).astype(np.int32)
    out = rows.copy()
    gsm.sort_rows(graphs[1000], out)
    np.testing.assert_array_equal(out, lex(rows))


def test_sort_extreme_ids(graphs):
    n = 1 << 25
    vals = np.array([0, 1, n - 2, n - 1, n // 2, (n // 2) - 1], np.int32)
    rng = np.random.default_rng(5)
    rows = vals[rng.integers(0, len(vals), (10_000, 16))].astype(np.int32)
    t = torch.from_numpy(rows.copy()).cuda()
    gsm.sort_rows(graphs[n], t)
    np.testing.assert_array_equal(t.cpu().numpy(), lex(rows))


def test_sort_rejects_bad_q(graphs):
    rows = np.zeros((4, 17), np.int32)
    with pytest.raises(gsm.GsmError):
        gsm.sort_rows(graphs[2], rows)


@pytest.fixture(scope="module")
def powerlaw():
    w = W.powerlaw()
    return w, gsm.Graph.from_workload(w.graph)


def test_sorted_rows_small_workload():
    w = W.small()
    G = gsm.Graph.from_workload(w.graph, validate=True)
    for qr in w.queries:
        Q = gsm.Query.from_workload(qr)
        c, r = oracle.match(w.graph, qr)
        cg, rg, _ = gsm.match(G, Q, rows="host", rows_cap=max(c, 1), sort_rows=True)
        assert cg == c, qr.name
        np.testing.assert_array_equal(rg, r)


@pytest.mark.parametrize("k,root", [(9, (0, 32, 1)), (10, (1, 32, 5)), (13, (0, 8, 2))])
def test_sorted_rows_powerlaw_device(powerlaw, k, root):
    w, G = powerlaw
    qr = w.queries[k]
    print("sorted powerlaw", k, root, flush=True)
    c, r = oracle.match(w.graph, qr, threads=8, root=root)
    assert 0 < c < 4_000_000
    Q = gsm.Query.from_workload(qr)
    out = torch.full((c, qr.q), -1, dtype=torch.int32, device="cuda")
    # a small budget so the rows come from many chunks before the sort
    cg, _, _ = gsm.match(G, Q, rows=out, root=root, sort_rows=True, budget=gsm.min_budget(G, Q) * 4)
    torch.cuda.synchronize()
    assert cg == c
    np.testing.assert_array_equal(out.cpu().numpy(), r)


def test_sorted_rows_truncated(powerlaw):
    w, G = powerlaw
    qr = w.queries[13]
    root = (0, 16, 3)
    c, r = oracle.match(w.graph, qr, threads=8, root=root)
    cap = max(1, c // 3)
    Q = gsm.Query.from_workload(qr)
    cg, rg, _ = gsm.match(G, Q, rows="host", rows_cap=cap, root=root, sort_rows=True)
    assert cg == c and rg.shape[0] == cap
    np.testing.assert_array_equal(rg, lex(rg))
    # every kept row is a distinct member of the full result set
    full = {tuple(x) for x in r.tolist()}
    kept = [tuple(x) for x in rg.tolist()]
    assert all(x in full for x in kept)
    assert len(set(kept)) == cap


def test_sort_with_emit_is_unsupported(powerlaw):
    w, G = powerlaw
    Q = gsm.Query.from_workload(w.queries[0])
    with pytest.raises(gsm.GsmError) as e:
        gsm.match(G, Q, emit=lambda rows: 0, sort_rows=True)
    assert e.value.status == 9


def messy_csr(n, edges, rng):
    """An adjacency listing each edge in one or both directions, some twice,
    with self-loops, rows in random order."""
    adj = [[] for _ in range(n)]
    for a, b in edges:
        mode = rng.integers(0, 4)
        if mode == 0:
            adj[a].append(b)
        elif mode == 1:
            adj[b].append(a)
        else:
            adj[a].append(b)
            adj[b].append(a)
        if mode == 3:
            adj[a].append(b)
    for v in rng.integers(0, n, max(1, n // 5)):
        adj[v].append(v)
    rp = np.zeros(n + 1, np.int64)
    col = []
    for v in range(n):
        row = list(adj[v])
        rng.shuffle(row)
        col.extend(row)
        rp[v + 1] = len(col)
    return rp, np.asarray(col, np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_strip_matches_clean_graph(seed):
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(2, 40))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.1, 0.5)), L, seed)
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    edges = [(int(a), int(b)) for a, b in zip(src, g.col) if a < b]
    rp, col = messy_csr(n, edges, rng)
    G = gsm.Graph(rp, col, g.labels, strip=True)
    assert G.info()["nnz"] == g.nnz
    qr = W.random_query(int(rng.integers(1, 5)), 0.3, L, seed + 3)
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(g, qr)
    cg, rg, _ = gsm.match(G, Q, rows="host", rows_cap=max(c, 1), sort_rows=True)
    assert cg == c
    np.testing.assert_array_equal(rg, r)
    # the stripped graph also passes validation
    gsm.Graph(rp, col, g.labels, strip=True, validate=True)


def test_strip_still_rejects_bad_ids():
    rp = np.array([0, 1, 2], np.int64)
    col = np.array([1, 5], np.int32)
    with pytest.raises(gsm.GsmError) as e:
        gsm.Graph(rp, col, strip=True)
    assert e.value.status == 2
