"""Pins of the CPU oracle against brute force, closed forms and invariants.

The oracle enumerates embeddings (injective, label-preserving, edge-preserving
maps; all automorphic images counted), the result of the paper's Alg. 1.
Nothing here compares the oracle with itself: every expected value comes from
brute force over all injective maps, a closed form, a textbook routine, or a
relation between two different inputs.
"""
import math

import numpy as np
import pytest

import oracle
from bruteforce import embeddings
from golden_io import automorphisms, query_of
from paper_2003_01527_amd import workloads as W


def complete_graph(n, labels=None):
    return W.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)], labels)


def cycle_graph(n):
    return W.from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def path_query(k):
    return query_of([(i, i + 1) for i in range(k - 1)])


def cycle_query(k):
    return query_of([(i, (i + 1) % k) for i in range(k)])


def adjacency(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[src, g.col] = 1
    return A


# ------------------------------------------------------ brute force (T1) --

@pytest.mark.parametrize("seed", range(600))
def test_oracle_equals_bruteforce(seed):
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.integers(1, 10))
    L = int(rng.integers(0, 4))
    g = W.random_graph(n, float(rng.uniform(0.2, 0.8)), L, seed)
    q = int(rng.integers(1, min(5, max(n, 1)) + 1))
    qr = W.random_query(q, float(rng.uniform(0.0, 0.6)), L, seed + 1)
    expect = embeddings(g, qr)
    cnt, rows = oracle.match(g, qr)
    assert cnt == expect.shape[0]
    np.testing.assert_array_equal(rows, expect)
    # all-core variant and count-only give the same
    cnt2, rows2 = oracle.match(g, qr, threads=3)
    assert cnt2 == cnt
    np.testing.assert_array_equal(rows2, expect)
    assert oracle.match(g, qr, rows=False)[0] == cnt


@pytest.mark.parametrize("seed", range(40))
def test_oracle_root_slices_partition(seed):
    """Root slices on a fixed query vertex split the embedding set exactly."""
    g = W.random_graph(9, 0.6, 2, 500 + seed)
    qr = W.random_query(4, 0.3, 2, 900 + seed)
    expect = embeddings(g, qr)
    mod = 3
    root_q = seed % qr.q
    parts = []
    for rem in range(mod):
        c, r = oracle.match(g, qr, root=(root_q, mod, rem))
        assert c == r.shape[0]
        assert all(oracle.slice_hash(int(v)) % mod == rem for v in r[:, root_q])
        parts.append(r)
    allr = oracle.sort_rows(np.concatenate(parts))
    np.testing.assert_array_equal(allr, expect)


def test_slice_hash_published_values():
    """splitmix64 first outputs from seed 0 (Vigna's reference generator):
    state advances by the golden-ratio constant before mixing, so the output of
    state 0 is the mix of 0x9E3779B97F4A7C15 = 0xE220A8397B1DCDAF."""
    assert oracle.slice_hash(0) == 0xE220A8397B1DCDAF
    assert oracle.slice_hash(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


# ------------------------------------------------------ closed forms (T2) --

@pytest.mark.parametrize("name,aut,edges", automorphisms())
def test_query_in_itself_gives_automorphisms(name, aut, edges):
    qr = query_of(edges)
    g = W.from_edges(qr.q, edges)
    assert oracle.match(g, qr, rows=False)[0] == aut


@pytest.mark.parametrize("name,aut,edges", automorphisms())
@pytest.mark.parametrize("n", [6, 8])
def test_any_query_in_complete_graph(name, aut, edges, n):
    qr = query_of(edges)
    if qr.q > n:
        pytest.skip("query larger than K_n")
    expect = math.factorial(n) // math.factorial(n - qr.q)
    assert oracle.match(complete_graph(n), qr, rows=False)[0] == expect


def test_triangle_in_complete_graph_closed_form():
    for n in range(3, 25):
        assert oracle.match(complete_graph(n), query_of([(0, 1), (1, 2), (0, 2)]), rows=False)[0] == \
            n * (n - 1) * (n - 2)


@pytest.mark.parametrize("seed", range(12))
def test_edge_triangle_c4_star_closed_forms(seed):
    g = W.random_graph(30, 0.25 + 0.03 * seed, 0, 77 + seed)
    A = adjacency(g)
    d = A.sum(1)
    m2 = int(d.sum())
    assert oracle.match(g, query_of([(0, 1)]), rows=False)[0] == m2
    A3 = A @ A @ A
    assert oracle.match(g, query_of([(0, 1), (1, 2), (0, 2)]), rows=False)[0] == int(np.trace(A3))
    c4 = int(np.trace(A3 @ A)) - 2 * int((d * d).sum()) + m2
    assert oracle.match(g, query_of([(0, 1), (1, 2), (2, 3), (0, 3)]), rows=False)[0] == c4
    for s in (2, 3, 4):
        star = query_of([(0, i) for i in range(1, s + 1)])
        expect = sum(math.perm(int(x), s) for x in d)
        assert oracle.match(g, star, rows=False)[0] == expect


@pytest.mark.parametrize("seed", range(6))
def test_labelled_star_closed_form(seed):
    g = W.random_graph(25, 0.35, 3, 300 + seed)
    A = adjacency(g)
    lab = g.labels
    # centre label 1, leaves labels (0, 0, 2)
    qr = query_of([(0, 1), (0, 2), (0, 3)], [1, 0, 0, 2])
    need = {0: 2, 2: 1}
    expect = 0
    for v in range(g.n):
        if lab[v] != 1:
            continue
        nb = np.nonzero(A[v])[0]
        prod = 1
        for l, s in need.items():
            prod *= math.perm(int((lab[nb] == l).sum()), s)
        expect += prod
    assert oracle.match(g, qr, rows=False)[0] == expect


@pytest.mark.parametrize("n", range(3, 10))
def test_paths_and_cycles_in_cycles(n):
    g = cycle_graph(n)
    for k in range(2, n + 1):
        assert oracle.match(g, path_query(k), rows=False)[0] == 2 * n
    for k in range(3, n):
        assert oracle.match(g, cycle_query(k), rows=False)[0] == 0
    assert oracle.match(g, cycle_query(n), rows=False)[0] == 2 * n


def test_path3_in_triangle_is_non_induced():
    g = complete_graph(3)
    assert oracle.match(g, path_query(3), rows=False)[0] == 6
    assert embeddings(g, path_query(3), induced=True).shape[0] == 0


def test_single_vertex_query_counts_label_class():
    g = W.random_graph(12, 0.3, 3, 5)
    for l in range(3):
        qr = W.Query(1, np.zeros((0, 2), np.int32), np.array([l], np.int32))
        c, r = oracle.match(g, qr)
        assert c == int((g.labels == l).sum())
        np.testing.assert_array_equal(r[:, 0], np.nonzero(g.labels == l)[0])


def test_disconnected_query_rejected():
    g = complete_graph(4)
    with pytest.raises(RuntimeError):
        oracle.match(g, query_of([(0, 1), (2, 3)]))


# ---------------------------------------------------------- metamorphic (T3) --

@pytest.mark.parametrize("seed", range(20))
def test_vertex_permutation_maps_rows(seed):
    g = W.random_graph(40, 0.15, 2, 1000 + seed)
    qr = W.random_query(4, 0.3, 2, 2000 + seed)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.n)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    e = np.stack([perm[src], perm[g.col]], 1)
    lab = np.empty_like(g.labels)
    lab[perm] = g.labels
    gp = W.from_edges(g.n, e, lab)
    c, r = oracle.match(g, qr)
    cp, rp = oracle.match(gp, qr)
    assert c == cp
    np.testing.assert_array_equal(oracle.sort_rows(perm[r].astype(np.int32)), rp)


@pytest.mark.parametrize("seed", range(20))
def test_query_permutation_permutes_columns(seed):
    g = W.random_graph(40, 0.15, 2, 3000 + seed)
    qr = W.random_query(5, 0.3, 2, 4000 + seed)
    rng = np.random.default_rng(seed)
    sigma = rng.permutation(qr.q)   # new id of old vertex u is sigma[u]
    q2 = W.Query(qr.q, sigma[qr.edges].astype(np.int32), np.empty_like(qr.labels))
    q2.labels[sigma] = qr.labels
    c, r = oracle.match(g, qr)
    c2, r2 = oracle.match(g, q2)
    assert c == c2
    back = np.empty_like(r2)
    back[:, :] = r2[:, sigma]   # column u of the old query is column sigma[u]
    np.testing.assert_array_equal(oracle.sort_rows(back), r)


@pytest.mark.parametrize("seed", range(10))
def test_disjoint_union_and_isolated_vertices(seed):
    g1 = W.random_graph(20, 0.3, 2, 5000 + seed)
    g2 = W.random_graph(15, 0.35, 2, 6000 + seed)
    qr = W.random_query(4, 0.3, 2, 7000 + seed)
    src1 = np.repeat(np.arange(g1.n), np.diff(g1.row_ptr))
    src2 = np.repeat(np.arange(g2.n), np.diff(g2.row_ptr))
    e = np.concatenate([np.stack([src1, g1.col], 1), np.stack([src2 + g1.n, g2.col + g1.n], 1)])
    iso = 5
    lab = np.concatenate([g1.labels, g2.labels, np.zeros(iso, np.int32)])
    gu = W.from_edges(g1.n + g2.n + iso, e, lab)
    c1 = oracle.match(g1, qr, rows=False)[0]
    c2 = oracle.match(g2, qr, rows=False)[0]
    assert oracle.match(gu, qr, rows=False)[0] == c1 + c2


def test_walk_queries_contain_their_source_map():
    w = W.small()
    for qr in w.queries:
        c, r = oracle.match(w.graph, qr)
        assert c == r.shape[0] > 0
        hit = np.all(r == qr.source[None, :], axis=1)
        assert hit.any(), qr.name


# ---------------------------------------------------- textbook triangles --

@pytest.mark.parametrize("seed", range(10))
def test_forward_triangle_count_matches_trace_and_oracle(seed):
    g = W.random_graph(60, 0.1 + 0.02 * seed, 0, 8000 + seed)
    A = adjacency(g)
    t = oracle.triangles(g, threads=2)
    assert 6 * t == int(np.trace(A @ A @ A))
    assert oracle.match(g, query_of([(0, 1), (1, 2), (0, 2)]), rows=False)[0] == 6 * t
