"""Error paths under injected device-allocation failures: every failing call
returns GSM_E_OOM, and once allocations are allowed again the same graph and
workspace give the oracle's results."""
import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def lift_limit():
    yield
    gsm.testing_fail_allocations(-1)


def test_graph_create_fails_cleanly_at_every_allocation():
    g = W.random_graph(60, 0.2, 3, 1)
    failed = 0
    for after in range(0, 16):
        gsm.testing_fail_allocations(after)
        try:
            G = gsm.Graph.from_workload(g)
            G.close()
        except gsm.GsmError as e:
            assert e.status == 4, e
            failed += 1
        finally:
            gsm.testing_fail_allocations(-1)
    assert failed > 0
    qr = W.random_query(4, 0.3, 3, 2)
    c, r = oracle.match(g, qr)
    G = gsm.Graph.from_workload(g)
    cg, rg, _ = gsm.match(G, gsm.Query.from_workload(qr), rows="host", rows_cap=max(c, 1), sort_rows=True)
    assert cg == c
    np.testing.assert_array_equal(rg, r)


def test_match_fails_cleanly_and_recovers():
    w = W.small()
    G = gsm.Graph.from_workload(w.graph)
    qr = w.queries[0]
    Q = gsm.Query.from_workload(qr)
    c, r = oracle.match(w.graph, qr)
    failed = 0
    for after in range(0, 30, 2):
        G2 = gsm.Graph.from_workload(w.graph)  # a fresh workspace, so the match allocates
        gsm.testing_fail_allocations(after)
        try:
            cg, rg, _ = gsm.match(G2, Q, rows="host", rows_cap=max(c, 1), sort_rows=True,
                                  budget=gsm.min_budget(G2, Q, host_rows=True) + 4096)
            gsm.testing_fail_allocations(-1)
            assert cg == c
            np.testing.assert_array_equal(rg, r)
        except gsm.GsmError as e:
            gsm.testing_fail_allocations(-1)
            assert e.status == 4, e
            failed += 1
            # the same graph and workspace work again
            cg, rg, _ = gsm.match(G2, Q, rows="host", rows_cap=max(c, 1), sort_rows=True)
            assert cg == c
            np.testing.assert_array_equal(rg, r)
        G2.close()
    assert failed > 0
    assert gsm.match(G, Q)[0] == c


def test_batch_fails_cleanly_and_recovers():
    w = W.small()
    Qs = [gsm.Query.from_workload(q) for q in w.queries]
    expect = [oracle.match(w.graph, q, rows=False)[0] for q in w.queries]
    for after in (0, 3, 6):
        G2 = gsm.Graph.from_workload(w.graph)
        gsm.testing_fail_allocations(after)
        try:
            got = gsm.match_batch(G2, Qs).tolist()
            gsm.testing_fail_allocations(-1)
            assert got == expect
        except gsm.GsmError as e:
            gsm.testing_fail_allocations(-1)
            assert e.status == 4, e
            assert gsm.match_batch(G2, Qs).tolist() == expect
        G2.close()
