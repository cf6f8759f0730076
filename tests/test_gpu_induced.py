"""Induced semantics (GSM_MATCH_INDUCED) against the oracle's induced option
(itself pinned by brute force, closed forms and complementation)."""
import os
from math import perm

import numpy as np
import pytest

import oracle
from golden_io import automorphisms, query_of
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def gpu_sorted(G, Q, **kw):
    c, _, _ = gsm.match(G, Q, induced=True, **kw)
    c2, rows, _ = gsm.match(G, Q, rows="host", rows_cap=max(c, 1), induced=True, sort_rows=True, **kw)
    assert c2 == c
    return c, rows


@pytest.mark.parametrize("seed", range(80))
def test_random_instances_induced(seed):
    rng = np.random.default_rng(99_000 + seed)
    n = int(rng.integers(2, 40))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.1, 0.8)), L, seed)
    qr = W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0, 0.7)), L, seed + 9)
    G = gsm.Graph.from_workload(g, validate=True)
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(g, qr, induced=True)
    cg, rg = gpu_sorted(G, Q, filter_rounds=seed % 3, lookahead=bool(seed % 2))
    assert cg == c
    np.testing.assert_array_equal(rg, r)
    if seed % 4 == 0:
        aut, _ = gsm.symmetry(Q)
        cu, _, _ = gsm.match(G, Q, induced=True, unique=True)
        assert cu * aut == c


@pytest.mark.parametrize("name,aut,edges", automorphisms())
def test_shapes_in_complete_graph_induced(name, aut, edges):
    n = 9
    qr = query_of(edges, name=name)
    g = W.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    G = gsm.Graph.from_workload(g)
    c, _, _ = gsm.match(G, gsm.Query.from_workload(qr), induced=True)
    complete = len(edges) == qr.q * (qr.q - 1) // 2
    assert c == (perm(n, qr.q) if complete else 0)


@pytest.fixture(scope="module")
def powerlaw():
    w = W.powerlaw()
    return w, gsm.Graph.from_workload(w.graph)


@pytest.mark.parametrize("k", [0, 3, 6, 9, 12, 15, 18])
def test_powerlaw_slices_induced(powerlaw, k):
    w, G = powerlaw
    qr = w.queries[k]
    Q = gsm.Query.from_workload(qr)
    root = (k % qr.q, 64, (k + 3) % 11)
    print("induced powerlaw", k, root, flush=True)
    c, _ = oracle.match(w.graph, qr, rows=False, threads=NCPU, root=root, induced=True)
    cg, _, _ = gsm.match(G, Q, root=root, induced=True)
    assert cg == c


def test_powerlaw_rows_induced(powerlaw):
    w, G = powerlaw
    qr = w.queries[13]
    root = (0, 8, 2)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root, induced=True)
    Q = gsm.Query.from_workload(qr)
    cg, rg = gpu_sorted(G, Q, root=root, budget=gsm.min_budget(G, Q, host_rows=True) + (1 << 18))
    assert cg == c
    np.testing.assert_array_equal(rg, r)


@pytest.mark.parametrize("name", ["P3", "P4", "C4", "star3", "paw", "house_tail"])
def test_unlabelled_rmat_shapes_induced(name):
    g = W.rmat_graph(9, 4, 0.57, 0.19, 0.19, 31)
    qr = W.shape(name)
    G = gsm.Graph.from_workload(g)
    c, _ = oracle.match(g, qr, rows=False, threads=NCPU, induced=True)
    cg, _, _ = gsm.match(G, gsm.Query.from_workload(qr), induced=True)
    assert cg == c
