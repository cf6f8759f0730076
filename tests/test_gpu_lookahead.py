"""One-step look-ahead (GSM_MATCH_LOOKAHEAD) against the oracle.

The look-ahead only prunes rows that cannot be extended to an embedding, so
counts and row sets must equal the oracle's exactly, and no level may hold
more rows than without it.  Cases cover the label-grouped adjacency table,
graphs with too many labels for it, and unlabelled graphs.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def sorted_rows(G, Q, **kw):
    cnt, _, _ = gsm.match(G, Q, **kw)
    c2, rows, _ = gsm.match(G, Q, rows="host", rows_cap=max(cnt, 1), sort_rows=True, **kw)
    assert c2 == cnt
    return cnt, rows


@pytest.mark.parametrize("seed", range(80))
def test_random_instances_with_lookahead(seed):
    rng = np.random.default_rng(77_000 + seed)
    n = int(rng.integers(2, 48))
    # 0: unlabelled, 1-3: few labels, 100: no label table
    L = [0, 1, 2, 3, 100][seed % 5]
    g = W.random_graph(n, float(rng.uniform(0.1, 0.7)), L, seed)
    qr = W.random_query(int(rng.integers(2, 7)), float(rng.uniform(0, 0.6)), min(L, 3), seed + 11)
    G = gsm.Graph.from_workload(g, validate=True)
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(g, qr)
    cg, rg = sorted_rows(G, Q, lookahead=True, filter_rounds=seed % 3)
    assert cg == c
    np.testing.assert_array_equal(rg, r)


def test_small_workload_with_lookahead():
    w = W.small()
    G = gsm.Graph.from_workload(w.graph, validate=True)
    for qr in w.queries:
        Q = gsm.Query.from_workload(qr)
        c, r = oracle.match(w.graph, qr)
        cg, rg = sorted_rows(G, Q, lookahead=True)
        assert cg == c, qr.name
        np.testing.assert_array_equal(rg, r)


@pytest.fixture(scope="module")
def powerlaw():
    w = W.powerlaw()
    return w, gsm.Graph.from_workload(w.graph)


@pytest.mark.parametrize("k", range(20))
def test_powerlaw_slices_with_lookahead(powerlaw, k):
    w, G = powerlaw
    qr = w.queries[k]
    Q = gsm.Query.from_workload(qr)
    root = ((k + 1) % qr.q, 64, (k + 2) % 7)
    print("powerlaw lookahead slice", k, root, flush=True)
    c, _ = oracle.match(w.graph, qr, rows=False, threads=NCPU, root=root)
    cg, _, st = gsm.match(G, Q, root=root, lookahead=True)
    assert cg == c
    _, _, st0 = gsm.match(G, Q, root=root)
    for i in range(qr.q):
        assert st["rows"][i] <= st0["rows"][i]
    assert st["rows"][qr.q - 1] == c


def test_powerlaw_rows_with_lookahead_and_small_budget(powerlaw):
    w, G = powerlaw
    qr = w.queries[13]
    root = (0, 8, 2)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root)
    Q = gsm.Query.from_workload(qr)
    budget = gsm.min_budget(G, Q, host_rows=True) + (1 << 18)
    cg, rg = sorted_rows(G, Q, root=root, lookahead=True, budget=budget)
    assert cg == c
    np.testing.assert_array_equal(rg, r)


def test_lookahead_prunes_on_powerlaw(powerlaw):
    """Some level holds strictly fewer rows with the look-ahead."""
    w, G = powerlaw
    fewer = 0
    for qr in w.queries[:8]:
        Q = gsm.Query.from_workload(qr)
        root = (0, 16, 1)
        c1, _, s1 = gsm.match(G, Q, root=root, lookahead=True)
        c0, _, s0 = gsm.match(G, Q, root=root)
        assert c1 == c0
        fewer += sum(s1["rows"][i] < s0["rows"][i] for i in range(qr.q))
    assert fewer > 0


@pytest.mark.parametrize("name", ["K3", "K4", "C5", "house_tail"])
def test_shapes_on_unlabelled_rmat_with_lookahead(name):
    g = W.rmat_graph(9, 4, 0.57, 0.19, 0.19, 31)
    qr = W.shape(name)
    G = gsm.Graph.from_workload(g)
    c, _ = oracle.match(g, qr, rows=False, threads=NCPU)
    cg, _, _ = gsm.match(G, gsm.Query.from_workload(qr), lookahead=True)
    assert cg == c


# --- two-step look-ahead (GSM_MATCH_LOOKAHEAD2) ---

@pytest.mark.parametrize("seed", range(60))
def test_random_instances_with_two_step_lookahead(seed):
    rng = np.random.default_rng(79_000 + seed)
    n = int(rng.integers(2, 48))
    L = [1, 2, 3, 4, 0][seed % 5]
    g = W.random_graph(n, float(rng.uniform(0.1, 0.6)), L, seed)
    qr = W.random_query(int(rng.integers(2, 7)), float(rng.uniform(0, 0.6)), L, seed + 13)
    G = gsm.Graph.from_workload(g, validate=True)
    Q = gsm.Query.from_workload(qr)
    kw = {} if oracle.match(g, qr, rows=False)[0] <= 300_000 else {"root": (0, 64, seed % 64)}
    c, r = oracle.match(g, qr, **kw)
    cg, rg = sorted_rows(G, Q, lookahead2=True, filter_rounds=seed % 3, **kw)
    assert cg == c
    np.testing.assert_array_equal(rg, r)


@pytest.mark.parametrize("k", range(0, 20, 2))
def test_powerlaw_slices_with_two_step_lookahead(powerlaw, k):
    w, G = powerlaw
    qr = w.queries[k]
    Q = gsm.Query.from_workload(qr)
    root = ((k + 1) % qr.q, 64, (k + 5) % 11)
    c, _ = oracle.match(w.graph, qr, rows=False, threads=NCPU, root=root)
    c2, _, s2 = gsm.match(G, Q, root=root, lookahead2=True)
    c1, _, s1 = gsm.match(G, Q, root=root, lookahead=True)
    print("powerlaw two-step slice", k, root, c, [s1["rows"][i] - s2["rows"][i] for i in range(qr.q)], flush=True)
    assert c2 == c1 == c
    for i in range(qr.q):
        assert s2["rows"][i] <= s1["rows"][i]


def test_two_step_lookahead_rows_small_budget(powerlaw):
    w, G = powerlaw
    qr = w.queries[4]
    root = (0, 16, 3)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root)
    Q = gsm.Query.from_workload(qr)
    budget = gsm.min_budget(G, Q, host_rows=True) + (4 << 20)
    cg, rg = sorted_rows(G, Q, root=root, lookahead2=True, budget=budget)
    assert cg == c
    np.testing.assert_array_equal(rg, r)
