"""The seeded generators: deterministic, and graphs are simple, symmetric and sorted."""
import numpy as np

from paper_2003_01527_amd import workloads as W


def check_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.shape[0]
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col >= 0) and np.all(col < g.n)
    assert np.all(src != col)
    # strictly ascending within rows
    same = src[1:] == src[:-1]
    assert np.all(col[1:][same] > col[:-1][same])
    # symmetric
    fwd = np.sort(src.astype(np.int64) * g.n + col)
    rev = np.sort(col.astype(np.int64) * g.n + src)
    np.testing.assert_array_equal(fwd, rev)


def test_er_exact_size_and_deterministic():
    a = W.er_graph(1000, 4000, 7)
    b = W.er_graph(1000, 4000, 7)
    check_csr(a)
    assert a.nnz == 8000
    np.testing.assert_array_equal(a.col, b.col)
    assert not np.array_equal(a.col, W.er_graph(1000, 4000, 8).col)


def test_rmat_valid_and_deterministic():
    a = W.rmat_graph(12, 8.0, 0.57, 0.19, 0.19, 3)
    b = W.rmat_graph(12, 8.0, 0.57, 0.19, 0.19, 3)
    check_csr(a)
    np.testing.assert_array_equal(a.col, b.col)
    d = a.degrees()
    assert d.max() > 20 * d.mean()   # skewed degrees


def test_zipf_label_frequencies():
    lab = W.labels_zipf(200_000, 16, 1.0, 11)
    p = np.bincount(lab, minlength=16) / lab.shape[0]
    h = sum(1.0 / (k + 1) for k in range(16))
    expect = np.array([1.0 / ((k + 1) * h) for k in range(16)])
    assert np.all(np.abs(p - expect) < 0.005)


def test_small_workload_queries():
    w = W.small()
    check_csr(w.graph)
    names = [q.name for q in w.queries]
    assert names.count("paw") == 3 and names.count("P4") == 3
    assert names.count("C4") == 2 and names.count("star3") == 2
    for q in w.queries:
        lab = w.graph.labels
        assert np.array_equal(q.labels, lab[q.source])
        for a, b in q.edges.tolist():
            s, t = q.source[a], q.source[b]
            assert t in w.graph.col[w.graph.row_ptr[s]:w.graph.row_ptr[s + 1]]


def test_powerlaw_queries_shape_and_cap():
    w = W.powerlaw()
    check_csr(w.graph)
    assert len(w.queries) == 20
    for q in w.queries:
        assert 5 <= q.q <= 6 and 5 <= q.ne <= 9
        assert 0 < q.bound <= 2 ** 32
        assert abs(W.tree_hom_bound(w.graph, q) - q.bound) <= 1e-9 * q.bound
