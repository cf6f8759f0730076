"""Pins of the oracle's induced option (non-adjacent query vertices map to
non-adjacent data vertices): brute force over all injective maps, closed forms
in complete graphs and cycles, containment in the non-induced result, and
complementation (an induced embedding of Q in G is one of the complement of Q
in the complement of G)."""
from math import perm

import numpy as np
import pytest

import oracle
from bruteforce import embeddings
from golden_io import automorphisms, query_of
from paper_2003_01527_amd import workloads as W


@pytest.mark.parametrize("seed", range(150))
def test_induced_equals_bruteforce(seed):
    rng = np.random.default_rng(31_000 + seed)
    n = int(rng.integers(1, 8))
    L = int(rng.integers(0, 3))
    g = W.random_graph(n, float(rng.uniform(0.1, 0.9)), L, seed)
    qr = W.random_query(int(rng.integers(1, 5)), float(rng.uniform(0, 0.8)), L, seed + 1)
    c, r = oracle.match(g, qr, induced=True)
    b = embeddings(g, qr, induced=True)
    assert c == b.shape[0]
    np.testing.assert_array_equal(r, b)


@pytest.mark.parametrize("name,aut,edges", automorphisms())
@pytest.mark.parametrize("n", [5, 7])
def test_shapes_in_complete_graph_induced(name, aut, edges, n):
    qr = query_of(edges, name=name)
    g = W.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    complete = len(edges) == qr.q * (qr.q - 1) // 2
    c, _ = oracle.match(g, qr, rows=False, induced=True)
    assert c == (perm(n, qr.q) if complete and qr.q <= n else 0)


@pytest.mark.parametrize("n", [4, 5, 7, 9])
def test_paths_and_cycles_in_cycles_induced(n):
    g = W.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    for k in range(2, n + 1):
        path = query_of([(i, i + 1) for i in range(k - 1)])
        assert oracle.match(g, path, rows=False, induced=True)[0] == (2 * n if k < n else 0)
    cyc = query_of([(i, (i + 1) % n) for i in range(n)])
    assert oracle.match(g, cyc, rows=False, induced=True)[0] == 2 * n


def test_path3_in_triangle_is_not_induced():
    g = W.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    assert oracle.match(g, W.shape("P3"), rows=False)[0] == 6
    assert oracle.match(g, W.shape("P3"), rows=False, induced=True)[0] == 0


@pytest.mark.parametrize("seed", range(40))
def test_induced_rows_are_a_subset(seed):
    rng = np.random.default_rng(32_000 + seed)
    g = W.random_graph(int(rng.integers(5, 30)), float(rng.uniform(0.1, 0.6)), 2, seed)
    qr = W.random_query(int(rng.integers(2, 6)), float(rng.uniform(0, 0.6)), 2, seed + 2)
    _, ri = oracle.match(g, qr, induced=True)
    _, rn = oracle.match(g, qr)
    full = {tuple(x) for x in rn.tolist()}
    assert all(tuple(x) in full for x in ri.tolist())
    if qr.ne == qr.q * (qr.q - 1) // 2:
        np.testing.assert_array_equal(ri, rn)


def complement_graph(g):
    n = g.n
    A = np.zeros((n, n), dtype=bool)
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    A[src, g.col] = True
    iu = np.triu_indices(n, 1)
    keep = ~A[iu]
    return W.from_edges(n, np.stack([iu[0][keep], iu[1][keep]], 1), g.labels)


def connected(q, edges):
    seen, stack = {0}, [0]
    adj = {u: set() for u in range(q)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    while stack:
        u = stack.pop()
        for w in adj[u] - seen:
            seen.add(w)
            stack.append(w)
    return len(seen) == q


@pytest.mark.parametrize("seed", range(60))
def test_induced_count_survives_complementation(seed):
    rng = np.random.default_rng(33_000 + seed)
    for _ in range(50):
        qr = W.random_query(int(rng.integers(2, 6)), float(rng.uniform(0.2, 0.8)), 2, int(rng.integers(1 << 30)))
        E = {frozenset(e) for e in qr.edges.tolist()}
        cE = [(a, b) for a in range(qr.q) for b in range(a + 1, qr.q) if frozenset((a, b)) not in E]
        if cE and connected(qr.q, cE):
            break
    else:
        pytest.skip("no query with a connected complement drawn")
    cq = W.Query(qr.q, np.array(cE, np.int32), qr.labels, None, -1.0, "complement")
    g = W.random_graph(int(rng.integers(5, 25)), float(rng.uniform(0.2, 0.8)), 2, seed)
    ci, ri = oracle.match(g, qr, induced=True)
    cc, rc = oracle.match(complement_graph(g), cq, induced=True)
    assert ci == cc
    np.testing.assert_array_equal(ri, rc)
