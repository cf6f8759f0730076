"""The serving engine: every result equals the query matched alone (tolerance
zero: the work is integer), under concurrency, memory admission and timeouts."""
import numpy as np
import pytest

from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    w = W.batch(nq=96)
    G = gsm.Graph.from_workload(w.graph)
    Qs = [gsm.Query.from_workload(q) for q in w.queries]
    alone = [gsm.match(G, Q)[0] for Q in Qs]
    return w, G, Qs, alone


@pytest.mark.parametrize("workers,arena", [(1, 0), (2, 0), (4, 2 << 30), (3, 256 << 20)])
def test_results_equal_alone(setup, workers, arena):
    w, G, Qs, alone = setup
    srv = gsm.Server(G, workers=workers, arena_bytes=arena, max_batch=16)
    order = np.random.default_rng(workers).permutation(len(Qs))
    tickets = [(k, srv.submit(Qs[k])) for k in order.tolist()]
    res = {k: srv.wait(t) for k, t in tickets}
    srv.close()
    for k, r in res.items():
        assert r["count"] == alone[k], k
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
        assert 1 <= r["batch_size"] <= 16


def test_batches_overlap_on_device(setup):
    """With two workers, some request of one batch runs while another batch runs."""
    w, G, Qs, alone = setup
    srv = gsm.Server(G, workers=2, max_batch=4)
    tickets = [(k, srv.submit(Qs[k])) for k in range(len(Qs))]
    res = [srv.wait(t) for _, t in tickets]
    srv.close()
    spans = sorted({(r["t_admit_ns"], r["t_done_ns"]) for r in res})
    overlap = any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    assert overlap


def test_wait_timeout_and_unknown_ticket(setup):
    w, G, Qs, alone = setup
    heavy = int(np.argmax(alone))
    srv = gsm.Server(G, workers=1)
    t = srv.submit(Qs[heavy])
    try:
        srv.wait(t, timeout_ms=0)
        finished_first = True
    except gsm.GsmError as e:
        assert e.status == 10
        finished_first = False
    if not finished_first:
        assert srv.wait(t)["count"] == alone[heavy]
    with pytest.raises(gsm.GsmError) as ei:
        srv.wait(123456789)
    assert ei.value.status == 1
    srv.close()


def test_queries_destroyed_after_submit(setup):
    w, G, Qs, alone = setup
    srv = gsm.Server(G, workers=2)
    tickets = []
    for k in range(8):
        q = gsm.Query.from_workload(w.queries[k])
        tickets.append((k, srv.submit(q)))
        q.close()  # the server holds its own copy
    for k, t in tickets:
        assert srv.wait(t)["count"] == alone[k]
    srv.close()
