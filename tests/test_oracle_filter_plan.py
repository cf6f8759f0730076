"""Pins of the oracle's filtering stage and visiting order.

Filter (Sec. 3.2 "filtering", Alg. 1 Filter_candidate_set): candidate sets are
pinned by soundness against brute force (every embedding's image of u is a
candidate of u, for every option), by monotonicity (more rounds or the NE test
only remove candidates), by the worked NE example in tests/golden, and by the
unlabelled fixpoint: repeating the degree refinement until nothing changes
leaves exactly the delta(Q)-core of G, computed here by textbook peeling.

Order (Alg. 1 PreCompute_on_CPUs): pinned by the hand-worked examples in
tests/golden/plan_examples.txt and by structural properties.
"""
from collections import deque

import numpy as np
import pytest

import oracle
from bruteforce import embeddings
from golden_io import ints, parse_edges, query_of, records
from paper_2003_01527_amd import workloads as W


@pytest.mark.parametrize("seed", range(150))
def test_filter_is_sound(seed):
    rng = np.random.default_rng(20_000 + seed)
    n = int(rng.integers(4, 10))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.2, 0.8)), L, seed)
    qr = W.random_query(int(rng.integers(2, 5)), 0.4, L, seed + 99)
    emb = embeddings(g, qr)
    for rounds in range(4):
        for use_deg, use_ne in ((False, False), (True, False), (True, True)):
            cm = oracle.filter(g, qr, rounds=rounds, use_deg=use_deg, use_ne=use_ne)
            for u in range(qr.q):
                assert np.all((cm[emb[:, u]] >> u) & 1), (rounds, use_deg, use_ne, u)


@pytest.mark.parametrize("seed", range(30))
def test_filter_monotone(seed):
    g = W.random_graph(60, 0.08, 2, 300 + seed)
    qr = W.random_query(5, 0.3, 2, 400 + seed)
    prev = None
    for rounds in range(5):
        a = oracle.filter(g, qr, rounds=rounds, use_ne=True)
        b = oracle.filter(g, qr, rounds=rounds, use_ne=False)
        assert np.all((a & ~b) == 0)          # NE only removes
        if prev is not None:
            assert np.all((a & ~prev) == 0)   # rounds only remove
        prev = a
    c = oracle.filter(g, qr, rounds=0, use_deg=False, use_ne=False)
    labels_ok = np.zeros(g.n, np.uint16)
    for u in range(qr.q):
        labels_ok |= ((g.labels == qr.labels[u]).astype(np.uint16) << u)
    np.testing.assert_array_equal(c, labels_ok)


def kcore(g, k):
    """Textbook peeling: repeatedly delete vertices of degree < k."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    alive = np.ones(g.n, bool)
    dq = deque(np.nonzero(deg < k)[0].tolist())
    for v in dq:
        alive[v] = False
    while dq:
        v = dq.popleft()
        for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
            if alive[w]:
                deg[w] -= 1
                if deg[w] < k:
                    alive[w] = False
                    dq.append(w)
    return alive


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("shape", ["K3", "C4", "K4", "house_tail"])
def test_unlabelled_refinement_fixpoint_is_core(seed, shape):
    g = W.random_graph(200, 0.02 + 0.005 * seed, 0, 600 + seed)
    qr = W.shape(shape)
    delta = int(np.bincount(qr.edges.ravel(), minlength=qr.q).min())
    cm = oracle.filter(g, qr, rounds=g.n, use_ne=True)
    np.testing.assert_array_equal(cm != 0, kcore(g, delta))


def test_filter_ne_worked_example():
    rec = records("filter_ne_example.txt")[0]
    n = int(rec["n"][0])
    g = W.from_edges(n, parse_edges(rec["edges"]), ints(rec["labels"]))
    qr = query_of(parse_edges(rec["query_edges"]), ints(rec["query_labels"]))
    with_ne = oracle.filter(g, qr, rounds=0, use_ne=True)
    no_ne = oracle.filter(g, qr, rounds=0, use_ne=False)
    assert sorted(np.nonzero(with_ne & 1)[0].tolist()) == ints(rec["cand_q0_ne"])
    assert sorted(np.nonzero(no_ne & 1)[0].tolist()) == ints(rec["cand_q0_none"])
    for u in (1, 2, 3):
        assert sorted(np.nonzero((with_ne >> u) & 1)[0].tolist()) == ints(rec["cand_leaf"])
    assert oracle.match(g, qr, rows=False)[0] == int(rec["count"][0])


def test_filter_refinement_worked_example():
    rec = records("filter_refine_example.txt")[0]
    g = W.from_edges(int(rec["n"][0]), parse_edges(rec["edges"]))
    qr = query_of(parse_edges(rec["query_edges"]))
    for r in (0, 1, 2):
        got = oracle.filter(g, qr, rounds=r)
        assert got.tolist() == ints(rec["mask_r%d" % r]), r
    assert oracle.match(g, qr, rows=False)[0] == int(rec["count"][0])


@pytest.mark.parametrize("rec", records("plan_examples.txt"), ids=["A", "B"])
def test_plan_worked_examples(rec):
    ge = parse_edges(rec["graph_edges"])
    n = 1 + max(max(e) for e in ge)
    g = W.from_edges(n, ge, ints(rec["graph_labels"]))
    qr = query_of(parse_edges(rec["query_edges"]), ints(rec["query_labels"]))
    order, parent, back = oracle.plan(qr.q, qr.edges, qr.labels, g.labels, g.degrees())
    assert order == ints(rec["order"])
    assert parent == ints(rec["parent"])
    assert back == ints(rec["backmask"])


@pytest.mark.parametrize("seed", range(100))
def test_plan_is_connected_permutation(seed):
    g = W.random_graph(50, 0.1, 3, seed)
    qr = W.random_query(2 + seed % 9, 0.3, 3, 50 + seed)
    order, parent, back = oracle.plan(qr.q, qr.edges, qr.labels, g.labels, g.degrees())
    assert sorted(order) == list(range(qr.q))
    E = set(map(tuple, qr.edges.tolist()))
    adj = lambda a, b: (a, b) in E or (b, a) in E  # noqa: E731
    for i in range(1, qr.q):
        assert back[i] != 0 and parent[i] == (back[i] & -back[i]).bit_length() - 1
        for j in range(i):
            assert bool((back[i] >> j) & 1) == adj(order[i], order[j])
