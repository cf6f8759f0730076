"""Batched matching (many queries per launch) against per-query matching and
the oracle: counts must be identical (tolerance zero, the work is integer)."""
import os

import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def test_batch_small_workload_and_shapes():
    w = W.small()
    G = gsm.Graph.from_workload(w.graph)
    qrs = list(w.queries)
    qrs.append(W.Query(1, np.zeros((0, 2), np.int32), np.array([1], np.int32)))
    qrs.append(W.Query(2, np.array([[0, 1]], np.int32), np.array([0, 2], np.int32)))
    qrs.append(W.Query(3, np.array([[0, 1], [1, 2], [0, 2]], np.int32), np.array([1, 1, 1], np.int32)))
    Qs = [gsm.Query.from_workload(q) for q in qrs]
    expect = [oracle.match(w.graph, q, rows=False)[0] for q in qrs]
    for rounds in (0, 1, 2):
        for heavy in (0, 1, 2 ** 64 - 1):
            got = gsm.match_batch(G, Qs, filter_rounds=rounds, batch_heavy_pairs=heavy)
            assert got.tolist() == expect, (rounds, heavy)


@pytest.mark.parametrize("seed", range(40))
def test_batch_random_instances(seed):
    rng = np.random.default_rng(90_000 + seed)
    L = int(rng.integers(0, 4))
    g = W.random_graph(int(rng.integers(5, 60)), float(rng.uniform(0.05, 0.5)), L, seed)
    qrs = [W.random_query(int(rng.integers(1, 7)), float(rng.uniform(0, 0.5)), L, seed * 100 + k)
           for k in range(int(rng.integers(1, 12)))]
    G = gsm.Graph.from_workload(g)
    Qs = [gsm.Query.from_workload(q) for q in qrs]
    expect = [oracle.match(g, q, rows=False)[0] for q in qrs]
    assert gsm.match_batch(G, Qs, filter_rounds=seed % 3).tolist() == expect
    assert gsm.match_batch(G, Qs, batch_heavy_pairs=2 ** 64 - 1).tolist() == expect
    assert gsm.match_batch(G, Qs, batch_heavy_pairs=1).tolist() == expect
    # small thresholds: queries leave the shared launches at deeper levels
    for heavy in (4, 16, 64):
        assert gsm.match_batch(G, Qs, batch_heavy_pairs=heavy).tolist() == expect, heavy


@pytest.fixture(scope="module")
def batch_workload():
    w = W.batch()
    G = gsm.Graph.from_workload(w.graph)
    Qs = [gsm.Query.from_workload(q) for q in w.queries]
    per = np.array([gsm.match(G, Q)[0] for Q in Qs], dtype=np.uint64)
    return w, G, Qs, per


@pytest.mark.parametrize("heavy", [0, 1, 2 ** 12, 2 ** 16, 2 ** 20, 2 ** 64 - 1])
def test_batch_equals_per_query_on_batch_workload(batch_workload, heavy):
    """Default split, every query on its own launches, every query shared, and
    thresholds that take queries out of the shared launches at deeper levels."""
    w, G, Qs, per = batch_workload
    got = gsm.match_batch(G, Qs, budget=64 << 30, batch_heavy_pairs=heavy)
    np.testing.assert_array_equal(got, per)


def test_batch_chunked_by_small_budget(batch_workload):
    w, G, Qs, per = batch_workload
    sub = list(range(0, 512, 8))
    got = gsm.match_batch(G, [Qs[k] for k in sub], budget=600 << 20)
    np.testing.assert_array_equal(got, per[sub])
    got = gsm.match_batch(G, [Qs[k] for k in sub], budget=600 << 20, batch_heavy_pairs=2 ** 14)
    np.testing.assert_array_equal(got, per[sub])


def test_batch_workload_small_queries_vs_oracle(batch_workload):
    w, G, Qs, per = batch_workload
    order = np.argsort(per)[:12]
    for k in order.tolist():
        c, _ = oracle.match(w.graph, w.queries[k], rows=False, threads=NCPU)
        assert int(per[k]) == c, k
