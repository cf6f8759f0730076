"""Query visiting order of the paper's host pre-computation.  TEST INFRASTRUCTURE ONLY.

Follows Sec. 3.2 (Alg. 1, PreCompute_on_CPUs): query vertices are taken
greedily by, in this priority, the largest node-mapping degree d_M (number of
edges to vertices already taken, a notion from VF3), the smallest probability
P_f of finding a compatible data vertex, then the largest degree; remaining
ties go to the smaller query id (the paper leaves them arbitrary).  P_f is the
independent-factor form the paper sketches: the frequency of the vertex's label
times the fraction of data vertices whose degree is at least the query vertex's
degree.  Both factors share the denominator n, so the comparison uses the exact
integer product  count(label) * count(deg >= d)  in place of P_f * n^2.

Every vertex after the first has d_M >= 1 (the query is connected), so the
order is a traversal of a spanning tree; a vertex's tree parent is its
earliest-ordered earlier neighbour, and its other earlier neighbours are the
non-tree edges checked during verification.
"""
from __future__ import annotations

import numpy as np


def plan(q, edges, qlabels, data_labels, data_degrees):
    """Returns (order, parent_pos, backmask) with positions in visiting order.

    order[i]      query vertex visited at position i
    parent_pos[i] position of its tree parent (-1 for i = 0)
    backmask[i]   bit j set when order[j] (j < i) is adjacent to order[i]
    """
    adj = [set() for _ in range(q)]
    for a, b in np.asarray(edges).reshape(-1, 2).tolist():
        adj[a].add(b)
        adj[b].add(a)
    ql = [0] * q if qlabels is None else [int(x) for x in qlabels]
    deg = np.sort(np.asarray(data_degrees, dtype=np.int64))
    n = deg.shape[0]
    if data_labels is None:
        def lab_count(l):
            return n if l == 0 else 0
    else:
        counts = np.bincount(np.asarray(data_labels, dtype=np.int64))

        def lab_count(l):
            return int(counts[l]) if l < counts.shape[0] else 0
    qdeg = [len(adj[u]) for u in range(q)]
    pf = [lab_count(ql[u]) * int(n - np.searchsorted(deg, qdeg[u], side="left")) for u in range(q)]
    dM = [0] * q
    order, left = [], set(range(q))
    while left:
        u = max(left, key=lambda x: (dM[x], -pf[x], qdeg[x], -x))
        order.append(u)
        left.remove(u)
        for w in adj[u]:
            if w in left:
                dM[w] += 1
    pos = {u: i for i, u in enumerate(order)}
    parent, back = [], []
    for i, u in enumerate(order):
        earlier = sorted(pos[w] for w in adj[u] if pos[w] < i)
        parent.append(earlier[0] if earlier else -1)
        back.append(sum(1 << j for j in earlier))
    return order, parent, back
