"""Brute force over all injective maps: the definition of an embedding, checked
map by map.  Independent of the oracle; tiny inputs only."""
import itertools

import numpy as np


def embeddings(g, qr, induced=False):
    n, q = g.n, qr.q
    A = np.zeros((n, n), dtype=bool)
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    A[src, g.col] = True
    if n < q:
        return np.zeros((0, q), dtype=np.int32)
    maps = np.array(list(itertools.permutations(range(n), q)), dtype=np.int64).reshape(-1, q)
    ok = np.ones(maps.shape[0], dtype=bool)
    gl = np.zeros(n, np.int64) if g.labels is None else np.asarray(g.labels, np.int64)
    ql = np.zeros(q, np.int64) if qr.labels is None else np.asarray(qr.labels, np.int64)
    for u in range(q):
        ok &= gl[maps[:, u]] == ql[u]
    E = set(map(tuple, np.asarray(qr.edges).reshape(-1, 2).tolist()))
    for a in range(q):
        for b in range(a + 1, q):
            if (a, b) in E or (b, a) in E:
                ok &= A[maps[:, a], maps[:, b]]
            elif induced:
                ok &= ~A[maps[:, a], maps[:, b]]
    qel = getattr(qr, "edge_labels", None)
    if qel is not None:
        # edge labels: the data edge's label (0 when the graph has none) must equal the query edge's
        EL = np.zeros((n, n), dtype=np.int64)
        gel = getattr(g, "edge_labels", None)
        if gel is not None:
            EL[src, g.col] = gel
        for (a, b), lab in zip(np.asarray(qr.edges).reshape(-1, 2).tolist(), np.asarray(qel).tolist()):
            ok &= EL[maps[:, a], maps[:, b]] == lab
    return maps[ok].astype(np.int32)  # permutations() is lexicographic: already sorted
