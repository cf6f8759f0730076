"""Adjacency bitmaps of high-degree vertices: edge checks against them are one
load instead of a list search, and every result is unchanged -- the oracle's
rows and counts on graphs with hubs, and equal counts with and without the
bitmaps on the 2^21-vertex graph's slices and the power-law workload."""
import os

import numpy as np
import pytest

import oracle
from paper_2003_01527_amd import gsm
from paper_2003_01527_amd import workloads as W

pytestmark = pytest.mark.gpu

NCPU = min(16, os.cpu_count() or 1)


def hub_graph(seed, n=20000, hubs=4, hub_deg=2100, extra=3):
    """Sparse random edges plus a few vertices of degree >= 2048 (hubs
    adjacent to each other too), labelled or not."""
    rng = np.random.default_rng(seed)
    E = [(int(a), int(b)) for a, b in rng.integers(0, n, (extra * n, 2))]
    H = rng.choice(n, hubs, replace=False)
    for h in H:
        E += [(int(h), int(v)) for v in rng.choice(n, hub_deg, replace=False)]
    E += [(int(a), int(b)) for a in H for b in H if a < b]
    return W.from_edges(n, E)


@pytest.mark.parametrize("seed", range(4))
def test_hub_graph_rows_equal_oracle(seed):
    g = hub_graph(seed)
    if seed % 2:
        g.labels = np.random.default_rng(seed).integers(0, 3, g.n).astype(np.int32)
    assert np.diff(g.row_ptr).max() >= 2048
    G = gsm.Graph.from_workload(g, validate=True)
    root = (0, 16, seed)
    for name in ("K3", "K4", "C4", "paw", "house_tail"):
        qr = W.shape(name)
        if g.labels is not None:
            qr.labels = np.zeros(qr.q, np.int32)
        Q = gsm.Query.from_workload(qr)
        listed = name != "house_tail"  # its slice has ~10^7 rows: counts only
        c, r = oracle.match(g, qr, rows=listed, threads=NCPU, root=root)
        cg, _, _ = gsm.match(G, Q, root=root)
        assert cg == c, name
        if listed:
            c2, rows, _ = gsm.match(G, Q, root=root, rows="host", rows_cap=max(c, 1))
            np.testing.assert_array_equal(oracle.sort_rows(rows), r)
        # and the same with the bitmaps off, and in batches
        if name in ("K4", "C4"):
            G0 = gsm.Graph.from_workload(g, hub_bitmaps=False)
            assert gsm.match(G0, Q, root=root)[0] == c
            assert gsm.match_batch(G, [Q, Q], root=root, batch_heavy_pairs=(1 << 64) - 1).tolist() == [c, c]


def test_large_graph_with_and_without_bitmaps():
    g = W.large_graph()
    G1 = gsm.Graph.from_workload(g)
    G0 = gsm.Graph.from_workload(g, hub_bitmaps=False)
    for name, root in (("K3", (0, 64, 5)), ("K4", (0, 2048, 3)), ("C5", (0, 1 << 18, 9)),
                       ("house_tail", (0, 1 << 20, 17))):
        Q = gsm.Query.from_workload(W.shape(name))
        c1 = gsm.match(G1, Q, root=root)[0]
        c0 = gsm.match(G0, Q, root=root)[0]
        print(name, root, c0, c1, flush=True)
        assert c1 == c0
    t = oracle.triangles(g, threads=NCPU)
    assert gsm.match(G1, gsm.Query.from_workload(W.shape("K3")), unique=True, budget=64 << 30)[0] == t
