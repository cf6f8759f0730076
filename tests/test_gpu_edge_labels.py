"""Edge labels (gsm_graph_create_ex, gsm_query_set_edge_labels) against the
oracle's edge-label option (pinned by brute force and the labelling partition
identity)."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def with_qlabels(qr, el):
    return W.Query(qr.q, qr.edges, qr.labels, None, -1.0, qr.name, np.asarray(el, np.int32))


def gpu_sorted(G, Q, **kw):
    c, _, _ = gsm.match(G, Q, **kw)
    c2, rows, _ = gsm.match(G, Q, rows="host", rows_cap=max(c, 1), sort_rows=True, **kw)
    assert c2 == c
    return c, rows


@pytest.mark.parametrize("seed", range(80))
def test_random_instances_edge_labels(seed):
    rng = np.random.default_rng(123_000 + seed)
    n = int(rng.integers(2, 40))
    L = [0, 1, 2, 3, 100][seed % 5]  # 100 labels: past the label table
    EL = int(rng.integers(1, 4))
    g = W.with_edge_labels(W.random_graph(n, float(rng.uniform(0.2, 0.8)), L, seed), EL, seed + 3)
    qr = W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0, 0.7)), min(L, 3), seed + 9)
    qr = with_qlabels(qr, rng.integers(0, EL, qr.ne))
    G = gsm.Graph.from_workload(g, validate=True)
    Q = gsm.Query.from_workload(qr)
    induced = bool(seed % 3 == 1)
    c, r = oracle.match(g, qr, induced=induced)
    cg, rg = gpu_sorted(G, Q, induced=induced, lookahead=bool(seed % 2), filter_rounds=seed % 3)
    assert cg == c
    np.testing.assert_array_equal(rg, r)
    aut, _ = gsm.symmetry(Q)
    cu, _, _ = gsm.match(G, Q, induced=induced, unique=True)
    assert cu * aut == c


def test_graph_without_edge_labels_means_label_zero():
    g = W.random_graph(30, 0.3, 2, 5)
    qr = W.random_query(4, 0.3, 2, 6)
    G = gsm.Graph.from_workload(g)
    for el in ([0] * qr.ne, [1] + [0] * (qr.ne - 1)):
        q2 = with_qlabels(qr, el)
        c, _ = oracle.match(g, q2, rows=False)
        cg, _, _ = gsm.match(G, gsm.Query.from_workload(q2))
        assert cg == c
    assert gsm.match(G, gsm.Query.from_workload(with_qlabels(qr, [1] * qr.ne)))[0] == 0


@pytest.fixture(scope="module")
def powerlaw_el():
    w = W.powerlaw()
    g = W.with_edge_labels(w.graph, 3, 77)
    return w, g, gsm.Graph.from_workload(g)


@pytest.mark.parametrize("k", [0, 4, 9, 13, 17])
def test_powerlaw_slices_edge_labels(powerlaw_el, k):
    w, g, G = powerlaw_el
    rng = np.random.default_rng(k)
    qr = with_qlabels(w.queries[k], rng.integers(0, 3, w.queries[k].ne))
    root = (k % qr.q, 16, k % 5)
    print("edge-labelled powerlaw", k, root, flush=True)
    c, r = oracle.match(g, qr, threads=NCPU, root=root)
    Q = gsm.Query.from_workload(qr)
    cg, rg = gpu_sorted(G, Q, root=root, budget=gsm.min_budget(G, Q, host_rows=True) + (1 << 20))
    assert cg == c
    np.testing.assert_array_equal(rg, r)


def test_device_pointer_graph_with_edge_labels():
    g = W.with_edge_labels(W.random_graph(25, 0.4, 2, 11), 2, 12)
    q0 = W.random_query(4, 0.4, 2, 13)
    qr = with_qlabels(q0, [k % 2 for k in range(q0.ne)])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    G = gsm.Graph(dev(g.row_ptr), dev(g.col), dev(g.labels), validate=True, edge_labels=dev(g.edge_labels))
    c, _ = oracle.match(g, qr, rows=False)
    assert gsm.match(G, gsm.Query.from_workload(qr))[0] == c


def test_asymmetric_edge_labels_rejected():
    g = W.from_edges(3, [(0, 1), (1, 2)])
    el = np.array([0, 1, 0, 0], np.int32)  # entries 0->1, 1->0, 1->2, 2->1: edge {0, 1} gets two labels
    with pytest.raises(gsm.GsmError) as e:
        gsm.Graph(g.row_ptr, g.col, edge_labels=el, validate=True)
    assert e.value.status == 2
    with pytest.raises(gsm.GsmError) as e:
        gsm.Graph(g.row_ptr, g.col, edge_labels=el, strip=True)
    assert e.value.status == 9


def test_batch_and_server_reject_edge_labelled_queries(powerlaw_el):
    w, g, G = powerlaw_el
    Qs = [gsm.Query.from_workload(with_qlabels(q, [0] * q.ne)) for q in w.queries[:2]]
    with pytest.raises(gsm.GsmError) as e:
        gsm.match_batch(G, Qs)
    assert e.value.status == 9
    srv = gsm.Server(G, workers=1)
    try:
        with pytest.raises(gsm.GsmError) as e:
            srv.submit(Qs[0])
        assert e.value.status == 9
    finally:
        srv.close()
