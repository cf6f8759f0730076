"""gsm_match_noalloc (no device allocation inside the call) against gsm_match,
through the C ABI: identical counts and identical row sets (integer work:
bit-exact), on two calls in a row with the second input smaller than the
first, with rows in device memory, host memory and a device-side callback.
"""
import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu


def _device_rows(fn, G, Q, q, **kw):
    import torch
    cnt, _, _ = fn(G, Q, **kw)
    buf = torch.full((max(cnt, 1), q), -1, dtype=torch.int32, device="cuda:0")
    c2, out, _ = fn(G, Q, rows=buf, **kw)
    torch.cuda.synchronize()
    assert c2 == cnt
    return cnt, oracle.sort_rows(out[:cnt].cpu().numpy())


def test_noalloc_equals_match_two_calls_second_smaller():
    import torch
    torch.cuda.init()
    # first call: the 2^17-vertex power-law graph, a 5-6 vertex query on a root
    # slice (several frontier chunks inside the fixed scratch)
    big = W.powerlaw()
    Gb = gsm.Graph.from_workload(big.graph)
    qr = big.queries[3]
    Qb = gsm.Query.from_workload(qr)
    print("call 1: powerlaw", qr.name, flush=True)
    kw = dict(root=(0, 8, 3))
    cn, rn = _device_rows(gsm.match_noalloc, Gb, Qb, qr.q, **kw)
    cm, rm = _device_rows(gsm.match, Gb, Qb, qr.q, **kw)
    assert cn == cm and cn > 0
    np.testing.assert_array_equal(rn, rm)
    # second call: the 1,000-vertex graph, a smaller input on the same scratch
    small = W.small()
    Gs = gsm.Graph.from_workload(small.graph)
    for qs in small.queries[:3]:
        print("call 2: small", qs.name, flush=True)
        Qs = gsm.Query.from_workload(qs)
        cn, rn = _device_rows(gsm.match_noalloc, Gs, Qs, qs.q)
        cm, rm = _device_rows(gsm.match, Gs, Qs, qs.q)
        assert cn == cm
        np.testing.assert_array_equal(rn, rm)
        # and both equal the oracle's rows
        co, ro = oracle.match(small.graph, qs)
        assert cn == co
        np.testing.assert_array_equal(rn, ro)


def test_noalloc_count_host_rows_and_callback():
    import torch
    torch.cuda.init()
    w = W.powerlaw()
    G = gsm.Graph.from_workload(w.graph)
    for k in (0, 7):
        qr = w.queries[k]
        Q = gsm.Query.from_workload(qr)
        print("count", qr.name, flush=True)
        kw = dict(root=(0, 4, 1))
        cn, _, _ = gsm.match_noalloc(G, Q, **kw)
        cm, _, _ = gsm.match(G, Q, **kw)
        assert cn == cm
        # rows through host memory (staging buffer inside the scratch)
        cap = min(cn, 1 << 20)
        c2, hn, _ = gsm.match_noalloc(G, Q, rows="host", rows_cap=cap, **kw)
        assert c2 == cn and hn.shape[0] == cap
        if cap == cn:
            _, hm, _ = gsm.match(G, Q, rows="host", rows_cap=cap, **kw)
            np.testing.assert_array_equal(oracle.sort_rows(hn), oracle.sort_rows(hm))
        # device-side callback: chunk sizes add up to the count
        seen = [0]

        def sink(ptr, nrows, q):
            seen[0] += nrows
            return False

        c3, _, _ = gsm.match_noalloc(G, Q, emit_device=sink, **kw)
        assert c3 == cn and seen[0] == cn


def test_noalloc_rejects_oversize_graph_and_sort():
    import torch
    torch.cuda.init()
    # a graph whose candidate masks and first frontier exceed the scratch
    n = 3_000_000
    g = W.from_edges(n, [(0, 1), (1, 2), (0, 2)])
    G = gsm.Graph.from_workload(g)
    Q = gsm.Query.from_workload(W.shape("K3"))
    with pytest.raises(gsm.GsmError) as ei:
        gsm.match_noalloc(G, Q)
    assert ei.value.status == 5 and "scratch" in str(ei.value)
    assert gsm.match(G, Q)[0] == 6
    small = W.small()
    Gs = gsm.Graph.from_workload(small.graph)
    Qs = gsm.Query.from_workload(small.queries[0])
    buf = torch.empty((4096, small.queries[0].q), dtype=torch.int32, device="cuda:0")
    with pytest.raises(gsm.GsmError) as ei:
        gsm.match_noalloc(Gs, Qs, rows=buf, sort_rows=True)
    assert ei.value.status == 9


def test_noalloc_on_degree_ordered_graph():
    # a graph stored renumbered by degree: rows still in the caller's ids,
    # equal to gsm_match's and the oracle's
    import torch
    torch.cuda.init()
    small = W.small()
    G = gsm.Graph.from_workload(small.graph, degree_order=True)
    for qs in small.queries[:3]:
        print("degree order:", qs.name, flush=True)
        Q = gsm.Query.from_workload(qs)
        cn, rn = _device_rows(gsm.match_noalloc, G, Q, qs.q)
        co, ro = oracle.match(small.graph, qs)
        assert cn == co
        np.testing.assert_array_equal(rn, ro)
