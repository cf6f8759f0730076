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


def test_runs_of_different_workers_overlap_on_device(setup):
    """Device time (HIP events on the workers' streams): some run of one
    worker executes while a run of another worker executes."""
    w, G, Qs, alone = setup
    srv = gsm.Server(G, workers=2, max_batch=4)
    tickets = [(k, srv.submit(Qs[k])) for k in range(len(Qs))]
    res = [srv.wait(t) for _, t in tickets]
    srv.close()
    for (k, _), r in zip(tickets, res):
        assert r["count"] == alone[k]
        assert 0 <= r["dev_start_ms"] <= r["dev_end_ms"]
    spans = {wk: sorted({(r["dev_start_ms"], r["dev_end_ms"]) for r in res if r["worker"] == wk}) for wk in (0, 1)}
    assert spans[0] and spans[1]
    overlap = any(a0 < b1 and b0 < a1 for a0, a1 in spans[0] for b0, b1 in spans[1])
    assert overlap


def test_arrivals_join_between_steps():
    """One worker: light queries that arrive while a heavy query is being
    expanded chunk by chunk start between its steps and finish before it,
    inside its device-time span."""
    import time
    g = W.powerlaw_graph()
    g.labels = None
    G = gsm.Graph.from_workload(g)
    heavy = gsm.Query.from_workload(W.shape("C4"))
    light = gsm.Query.from_workload(W.shape("K2"))
    c_heavy, c_light = gsm.match(G, heavy)[0], gsm.match(G, light)[0]
    # a small per-query reservation cuts the heavy query into many chunks
    srv = gsm.Server(G, workers=1, per_query_budget=24 << 20, batch_heavy_pairs=(1 << 64) - 1)
    th = srv.submit(heavy)
    time.sleep(0.05)
    tl = [srv.submit(light) for _ in range(4)]
    rh = srv.wait(th)
    rl = [srv.wait(t) for t in tl]
    srv.close()
    assert rh["count"] == c_heavy and all(r["count"] == c_light for r in rl)
    inside = [r for r in rl if r["t_done_ns"] < rh["t_done_ns"]]
    assert inside, "no light query finished before the heavy one"
    for r in inside:
        assert rh["dev_start_ms"] <= r["dev_start_ms"] <= r["dev_end_ms"] <= rh["dev_end_ms"]


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
