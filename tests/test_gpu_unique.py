"""Unique-subgraph mode (GSM_MATCH_UNIQUE) against the oracle.

The GPU rows must be exactly the oracle's embeddings that satisfy the query's
ordering constraints (one per class {f o s : s in Aut(Q)}, which the CPU tests
pin), and counts must equal the oracle count divided by |Aut(Q)|; on the
2^21-vertex graph the unique triangle count is the textbook triangle count.
Independently of the library's symmetry computation, the "one per subgraph"
tests take |Aut(Q)| by trying every permutation and check that the GPU's rows
are embeddings, that no two share an image (vertex set and edge set), and
that every image among the oracle's embeddings has one row.
"""
import itertools
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


# --- one embedding per subgraph, checked without the library's symmetry ---

def brute_aut(qr):
    """Automorphisms of a query by trying every permutation (q <= 7 here)."""
    q = qr.q
    E = {tuple(sorted(e)) for e in qr.edges.tolist()}
    lab = qr.labels if qr.labels is not None else np.zeros(q, np.int32)
    out = []
    for p in itertools.permutations(range(q)):
        if all(lab[p[u]] == lab[u] for u in range(q)) and {tuple(sorted((p[a], p[b]))) for a, b in E} == E:
            out.append(p)
    return out


def subgraph_keys(qr, rows):
    """Per row: its image vertex set and image edge set, as one sortable key.
    Two embeddings have equal keys iff they differ by an automorphism."""
    v = np.sort(rows, axis=1)
    e = qr.edges
    lo = np.minimum(rows[:, e[:, 0]], rows[:, e[:, 1]]).astype(np.int64)
    hi = np.maximum(rows[:, e[:, 0]], rows[:, e[:, 1]]).astype(np.int64)
    ek = np.sort(lo * (1 << 32) + hi, axis=1)
    return np.concatenate([v.astype(np.int64), ek], axis=1)


def as_void(a):
    """Rows as one opaque value each, so numpy set operations work row-wise."""
    a = np.ascontiguousarray(a)
    return a.view(np.dtype((np.void, a.dtype.itemsize * a.shape[1]))).ravel()


def check_one_per_subgraph(qr, oracle_rows, gpu_rows, aut):
    # every GPU row is an embedding of the slice
    assert np.isin(as_void(gpu_rows), as_void(oracle_rows)).all()
    kg = as_void(subgraph_keys(qr, gpu_rows))
    ko = as_void(subgraph_keys(qr, oracle_rows))
    # one row per subgraph, and every subgraph of the slice has one
    assert np.unique(kg).shape[0] == gpu_rows.shape[0]
    assert np.array_equal(np.unique(kg), np.unique(ko))
    assert gpu_rows.shape[0] * aut == oracle_rows.shape[0]


@pytest.mark.parametrize("root", [(2, 32, 1), (3, 32, 2), (4, 64, 5)])
def test_powerlaw_symmetric_query_one_per_subgraph(powerlaw, root):
    # the power-law query with a non-trivial automorphism group; the slice is
    # on a vertex every automorphism fixes, so all images of one subgraph
    # fall in the same slice
    w, G = powerlaw
    k = next(i for i, qr in enumerate(w.queries) if len(brute_aut(qr)) > 1)
    qr = w.queries[k]
    auts = brute_aut(qr)
    assert all(p[root[0]] == root[0] for p in auts)
    c, r = oracle.match(w.graph, qr, threads=NCPU, root=root)
    cg, rg = gpu_sorted(G, gsm.Query.from_workload(qr), root=root)
    print("powerlaw query", k, "|Aut|", len(auts), "slice", root, c, cg, flush=True)
    assert c > 0
    check_one_per_subgraph(qr, r, rg, len(auts))


@pytest.fixture(scope="module")
def rmat12():
    g = W.rmat_graph(12, 8, 0.57, 0.19, 0.19, 77)
    return g, gsm.Graph.from_workload(g)


# (shape, root slice on a vertex every automorphism fixes)
@pytest.mark.parametrize("name,root", [("paw", (0, 256, 3)), ("star3", (0, 4096, 9))])
def test_rmat_fixed_vertex_slice_one_per_subgraph(rmat12, name, root):
    g, G = rmat12
    qr = W.shape(name)
    auts = brute_aut(qr)
    assert all(p[root[0]] == root[0] for p in auts)
    c, r = oracle.match(g, qr, threads=NCPU, root=root)
    cg, rg = gpu_sorted(G, gsm.Query.from_workload(qr), root=root)
    print(name, "|Aut|", len(auts), root, c, cg, flush=True)
    assert c > 0
    check_one_per_subgraph(qr, r, rg, len(auts))


def test_rmat_triangles_one_per_subgraph(rmat12):
    g, G = rmat12
    qr = W.shape("K3")
    c, r = oracle.match(g, qr, threads=NCPU)
    cg, rg = gpu_sorted(G, gsm.Query.from_workload(qr))
    assert c > 0
    check_one_per_subgraph(qr, r, rg, len(brute_aut(qr)))


@pytest.mark.parametrize("name,scale", [("K4", 9), ("C4", 9), ("C5", 7), ("house_tail", 7)])
def test_small_rmat_one_per_subgraph(name, scale):
    g = W.rmat_graph(scale, 4, 0.57, 0.19, 0.19, 31)
    qr = W.shape(name)
    c, r = oracle.match(g, qr, threads=NCPU)
    cg, rg = gpu_sorted(gsm.Graph.from_workload(g), gsm.Query.from_workload(qr))
    assert c > 0
    check_one_per_subgraph(qr, r, rg, len(brute_aut(qr)))


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
