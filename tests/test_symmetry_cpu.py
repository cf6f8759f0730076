"""Query symmetry of the unique-subgraph mode (host code of the library, no
GPU): |Aut(Q)| and the ordering constraints f(a) < f(b).

Pins: the automorphism-group orders of tests/golden/automorphisms.txt; a brute
force over all vertex permutations of random labelled queries; and, against
the oracle's full embedding lists, that exactly one embedding of every class
{f o s : s in Aut(Q)} satisfies the constraints.  A class is identified by
the subgraph the embedding maps onto (image vertex set and image edge set):
two embeddings have the same image exactly when they differ by an
automorphism of the query.
"""
import itertools

import numpy as np
import pytest

import oracle
from golden_io import automorphisms, query_of
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W


def brute_aut(qr):
    q = qr.q
    lab = np.zeros(q, np.int64) if qr.labels is None else np.asarray(qr.labels)
    E = {frozenset(e) for e in np.asarray(qr.edges).reshape(-1, 2).tolist()}
    n = 0
    for p in itertools.permutations(range(q)):
        if all(lab[p[u]] == lab[u] for u in range(q)) and {frozenset((p[a], p[b])) for a, b in E} == E:
            n += 1
    return n


def satisfies(rows, pairs):
    ok = np.ones(rows.shape[0], dtype=bool)
    for a, b in pairs:
        ok &= rows[:, a] < rows[:, b]
    return ok


def image(row, edges):
    return (frozenset(row.tolist()), frozenset(frozenset((int(row[a]), int(row[b]))) for a, b in edges))


@pytest.mark.parametrize("name,aut,edges", automorphisms())
def test_aut_of_golden_shapes(name, aut, edges):
    qr = query_of(edges, name=name)
    got, pairs = gsm.symmetry(gsm.Query.from_workload(qr))
    assert got == aut, name
    assert len(pairs) <= qr.q * (qr.q - 1) // 2


@pytest.mark.parametrize("seed", range(60))
def test_aut_matches_brute_force(seed):
    rng = np.random.default_rng(5_000 + seed)
    q = int(rng.integers(1, 8))
    L = int(rng.integers(0, 3))
    qr = W.random_query(q, float(rng.uniform(0, 0.8)), L, seed)
    got, pairs = gsm.symmetry(gsm.Query.from_workload(qr))
    assert got == brute_aut(qr)
    if got == 1:
        assert pairs == []


def test_aut_of_large_symmetric_queries():
    # K_q: q!; the 16-vertex star: 15!; the 4x4 rook graph K4 x K4: 2 * 4!^2
    import math
    for q in (6, 8, 12, 16):
        e = [(a, b) for a in range(q) for b in range(a + 1, q)]
        assert gsm.symmetry(gsm.Query(q, e))[0] == math.factorial(q)
    assert gsm.symmetry(gsm.Query(16, [(0, k) for k in range(1, 16)]))[0] == math.factorial(15)
    rook = [(r * 4 + c, r * 4 + d) for r in range(4) for c in range(4) for d in range(c + 1, 4)]
    rook += [(r * 4 + c, s * 4 + c) for c in range(4) for r in range(4) for s in range(r + 1, 4)]
    assert gsm.symmetry(gsm.Query(16, rook))[0] == 2 * math.factorial(4) ** 2


@pytest.mark.parametrize("seed", range(80))
def test_one_embedding_per_class(seed):
    rng = np.random.default_rng(6_000 + seed)
    n = int(rng.integers(4, 22))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.2, 0.8)), L, seed)
    qr = W.random_query(int(rng.integers(2, 6)), float(rng.uniform(0.2, 0.9)), L, seed + 3)
    aut, pairs = gsm.symmetry(gsm.Query.from_workload(qr))
    c, rows = oracle.match(g, qr)
    assert c % aut == 0
    kept = rows[satisfies(rows, pairs)]
    assert kept.shape[0] * aut == c
    edges = np.asarray(qr.edges).reshape(-1, 2).tolist()
    imgs_all = {image(r, edges) for r in rows}
    imgs_kept = [image(r, edges) for r in kept]
    assert len(set(imgs_kept)) == len(imgs_kept) == len(imgs_all)


def test_shapes_in_complete_graph():
    # every q-subset of K_n is one subgraph per edge-set orbit: K4 in K7 = C(7,4)
    from math import comb
    g = W.from_edges(7, [(a, b) for a in range(7) for b in range(a + 1, 7)])
    qr = W.shape("K4")
    aut, pairs = gsm.symmetry(gsm.Query.from_workload(qr))
    c, rows = oracle.match(g, qr)
    assert satisfies(rows, pairs).sum() == comb(7, 4) == c // aut


def brute_aut_edge_labels(qr):
    q = qr.q
    lab = np.zeros(q, np.int64) if qr.labels is None else np.asarray(qr.labels)
    E = {frozenset(e): int(l) for e, l in zip(np.asarray(qr.edges).reshape(-1, 2).tolist(), qr.edge_labels)}
    n = 0
    for p in itertools.permutations(range(q)):
        if all(lab[p[u]] == lab[u] for u in range(q)) and \
                {frozenset((p[a], p[b])): l for (a, b), l in ((tuple(e), l) for e, l in E.items())} == E:
            n += 1
    return n


@pytest.mark.parametrize("seed", range(40))
def test_aut_with_edge_labels(seed):
    rng = np.random.default_rng(7_000 + seed)
    qr = W.random_query(int(rng.integers(2, 7)), float(rng.uniform(0.2, 0.9)), int(rng.integers(0, 2)), seed)
    qr.edge_labels = rng.integers(0, int(rng.integers(1, 3)), qr.ne).astype(np.int32)
    got, pairs = gsm.symmetry(gsm.Query.from_workload(qr))
    assert got == brute_aut_edge_labels(qr)
    g = W.with_edge_labels(W.random_graph(int(rng.integers(5, 16)), 0.5, 0 if qr.labels is None else 2, seed),
                           2, seed + 1)
    c, rows = oracle.match(g, qr)
    kept = rows[satisfies(rows, pairs)]
    assert kept.shape[0] * got == c
