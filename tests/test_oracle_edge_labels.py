"""Pins of the oracle's edge labels: brute force over all injective maps, and
the partition identity — every embedding of the edge-unlabelled query induces
exactly one labelling of the query's edges (the labels of the data edges it
maps them onto), so the counts over all L^|E(Q)| labellings sum to the
edge-unlabelled count, and the row sets partition its rows."""
import itertools

import numpy as np
import pytest

import oracle
from bruteforce import embeddings
from paper_2003_01527_amd import workloads as W


def labelled(qr, el):
    return W.Query(qr.q, qr.edges, qr.labels, None, -1.0, qr.name, np.asarray(el, np.int32))


@pytest.mark.parametrize("seed", range(120))
def test_edge_labels_equal_bruteforce(seed):
    rng = np.random.default_rng(41_000 + seed)
    n = int(rng.integers(1, 8))
    L = int(rng.integers(0, 3))
    EL = int(rng.integers(1, 4))
    g = W.with_edge_labels(W.random_graph(n, float(rng.uniform(0.2, 0.9)), L, seed), EL, seed + 1)
    qr = W.random_query(int(rng.integers(1, 5)), float(rng.uniform(0, 0.8)), L, seed + 2)
    qr = labelled(qr, rng.integers(0, EL, qr.ne))
    for induced in (False, True):
        c, r = oracle.match(g, qr, induced=induced)
        b = embeddings(g, qr, induced=induced)
        assert c == b.shape[0]
        np.testing.assert_array_equal(r, b)


@pytest.mark.parametrize("seed", range(30))
def test_labellings_partition_the_embeddings(seed):
    rng = np.random.default_rng(42_000 + seed)
    EL = int(rng.integers(1, 4))
    g = W.with_edge_labels(W.random_graph(int(rng.integers(6, 30)), float(rng.uniform(0.2, 0.6)), 2, seed), EL,
                           seed + 5)
    qr = W.random_query(int(rng.integers(2, 5)), float(rng.uniform(0, 0.5)), 2, seed + 6)
    if EL ** qr.ne > 243:
        pytest.skip("too many labellings")
    c_all, r_all = oracle.match(g, qr)
    total, rows = 0, []
    for el in itertools.product(range(EL), repeat=qr.ne):
        c, r = oracle.match(g, labelled(qr, el))
        total += c
        rows.append(r)
    assert total == c_all
    np.testing.assert_array_equal(oracle.sort_rows(np.concatenate(rows)), r_all)


def test_no_graph_edge_labels_means_label_zero():
    g = W.from_edges(4, [(0, 1), (1, 2), (2, 3), (0, 3)])
    c4 = W.shape("C4")
    assert oracle.match(g, labelled(c4, [0, 0, 0, 0]), rows=False)[0] == 8
    assert oracle.match(g, labelled(c4, [0, 1, 0, 0]), rows=False)[0] == 0


def test_triangles_by_colour():
    # K4 with edge {a, b} labelled (a + b) % 2: a triangle {x, y, z} has labels
    # x+y, y+z, x+z mod 2 — two odd and one even, or all even
    g = W.with_edge_labels(W.from_edges(4, [(a, b) for a in range(4) for b in range(a + 1, 4)]), 1, 0)
    src = np.repeat(np.arange(4), np.diff(g.row_ptr))
    g.edge_labels = ((src + g.col) % 2).astype(np.int32)
    k3 = W.shape("K3")  # edges 0-1, 1-2, 0-2
    counts = {el: oracle.match(g, labelled(k3, el), rows=False)[0] for el in itertools.product(range(2), repeat=3)}
    b = {el: embeddings(g, labelled(k3, el)).shape[0] for el in counts}
    assert counts == b
    assert sum(counts.values()) == 24
    assert counts[(0, 0, 0)] == 0  # no three vertices of one parity


@pytest.mark.parametrize("seed", range(10))
def test_generated_edge_labels_are_symmetric(seed):
    g = W.with_edge_labels(W.random_graph(40, 0.2, 2, seed), 5, seed)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lab = {(int(a), int(b)): int(l) for a, b, l in zip(src, g.col, g.edge_labels)}
    assert all(lab[(b, a)] == l for (a, b), l in lab.items())
    assert g.edge_labels.min() >= 0 and g.edge_labels.max() < 5


@pytest.mark.parametrize("seed", range(10))
def test_query_without_edge_labels_is_unconstrained(seed):
    rng = np.random.default_rng(43_000 + seed)
    g0 = W.random_graph(int(rng.integers(5, 25)), 0.4, 2, seed)
    g = W.with_edge_labels(g0, 3, seed + 1)
    qr = W.random_query(int(rng.integers(2, 5)), 0.4, 2, seed + 2)
    c0, r0 = oracle.match(g0, qr)
    c, r = oracle.match(g, qr)
    assert c == c0
    np.testing.assert_array_equal(r, r0)
