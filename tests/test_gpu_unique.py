"""Unique-subgraph mode (GSM_MATCH_UNIQUE) against the oracle.

The GPU rows must be exactly the oracle's embeddings that satisfy the query's
ordering constraints (one per class {f o s : s in Aut(Q)}, which the CPU tests
pin), and counts must equal the oracle count divided by |Aut(Q)|; on the
2^21-vertex graph the unique triangle count is the textbook triangle count.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def constrained(rows, pairs):
    ok = np.ones(rows.shape[0], dtype=bool)
    for a, b in pairs:
        ok &= rows[:, a] < rows[:, b]
    return rows[ok]


def gpu_sorted(G, Q, **kw):
    c, _, _ = gsm.match(G, Q, unique=True, **kw)
    c2, rows, _ = gsm.match(G, Q, rows="host", rows_cap=max(c, 1), unique=True, sort_rows=True, **kw)
    assert c2 == c
    return c, rows


@pytest.mark.parametrize("seed", range(60))
def test_random_instances_unique(seed):
    rng = np.random.default_rng(88_000 + seed)
    n = int(rng.integers(3, 40))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.2, 0.8)), L, seed)
    qr = W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0.2, 1.0)), L, seed + 5)
    G = gsm.Graph.from_workload(g, validate=True)
    Q = gsm.Query.from_workload(qr)
    aut, pairs = gsm.symmetry(Q)
    c, r = oracle.match(g, qr)
    cg, rg = gpu_sorted(G, Q, filter_rounds=seed % 3, lookahead=bool(seed % 2))
    assert cg * aut == c
    np.testing.assert_array_equal(rg, constrained(r, pairs))


@pytest.mark.parametrize("name", ["K3", "K4", "C4", "C5", "star3", "paw", "house_tail"])
def test_shapes_unique_on_rmat(name):
    g = W.rmat_graph(9, 4, 0.57, 0.19, 0.19, 31)
    qr = W.shape(name)
    G = gsm.Graph.from_workload(g)
    Q = gsm.Query.from_workload(qr)
    aut, pairs = gsm.symmetry(Q)
    c, _ = oracle.match(g, qr, rows=False, threads=NCPU)
    cg, _, _ = gsm.match(G, Q, unique=True)
    assert cg * aut == c


@pytest.fixture(scope="module")
def powerlaw():
    w = W.powerlaw()
    return w, gsm.Graph.from_workload(w.graph)


@pytest.mark.parametrize("k,root", [(9, (0, 32, 1)), (13, (0, 8, 2)), (10, (1, 32, 5))])
def test_powerlaw_slices_unique_rows(powerlaw, k, root):
    w, G = powerlaw
    qr = w.queries[k]
    Q = gsm.Query.from_workload(qr)
    aut, pairs = gsm.symmetry(Q)
    print("unique powerlaw", k, root, aut, flush=True)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root)
    expect = constrained(r, pairs)
    cg, rg = gpu_sorted(G, Q, root=root, budget=gsm.min_budget(G, Q, host_rows=True) + (1 << 20))
    assert cg == expect.shape[0]
    np.testing.assert_array_equal(rg, expect)


def test_large_unique_triangles():
    g = W.large_graph()
    G = gsm.Graph.from_workload(g)
    t = oracle.triangles(g, threads=NCPU)
    c, _, _ = gsm.match(G, gsm.Query.from_workload(W.shape("K3")), unique=True, budget=64 << 30)
    assert c == t


def test_batch_rejects_unique(powerlaw):
    w, G = powerlaw
    Qs = [gsm.Query.from_workload(q) for q in w.queries[:2]]
    with pytest.raises(gsm.GsmError) as e:
        gsm.match_batch(G, Qs, unique=True)
    assert e.value.status == 9
