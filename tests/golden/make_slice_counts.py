"""Writes the oracle's embedding counts on fixed root slices of the batching,
serving and large workloads (tests/golden/*_slice_counts.txt).

Only the CPU oracle (oracle/) and the seeded workload generators are called:
no value here comes from the HIP path.  Each file starts with a fingerprint
(SHA-1 over the graph's CSR arrays, labels and every query's edges and
labels) so a test can tell a changed generator from a wrong count.

A root slice keeps the embeddings f with splitmix64(f(r)) % mod == rem for a
query vertex r; slices of one query over all residues partition its
embeddings.

  python tests/golden/make_slice_counts.py [batch] [serving] [large]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2003_01527_amd import workloads as W  # noqa: E402

THREADS = os.cpu_count() or 1

# the slices the tests use
BATCH_SLICE = (0, 64, 0)             # every one of the 512 batching queries
SERVING_ARRIVALS = 256               # W.serving(nq=256): 256 arrivals, 256 distinct queries
SERVING_MOD = 64                     # arrival k counted on residue k % 64 of query vertex 0
LARGE_MOD = 1 << 20                  # large graph: residues chosen below
LARGE_SHAPES = ("C5", "house_tail", "K4")
LARGE_RESIDUES = 6


def fingerprint(g, queries) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(g.row_ptr, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(g.col, dtype=np.int32).tobytes())
    if g.labels is not None:
        h.update(np.ascontiguousarray(g.labels, dtype=np.int32).tobytes())
    for qr in queries:
        h.update(np.int32(qr.q).tobytes())
        h.update(np.ascontiguousarray(qr.edges, dtype=np.int32).tobytes())
        if qr.labels is not None:
            h.update(np.ascontiguousarray(qr.labels, dtype=np.int32).tobytes())
    return h.hexdigest()


def slice_hash_all(n: int) -> np.ndarray:
    """splitmix64 output for every vertex id (the finaliser of x + golden gamma)."""
    z = np.arange(n, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def write(fname, header, lines):
    with open(os.path.join(HERE, fname), "w") as f:
        for h in header:
            f.write("# " + h + "\n")
        for ln in lines:
            f.write(ln + "\n")
    print("wrote", fname, flush=True)


def make_batch():
    w = W.batch()
    t = time.time()
    lines = []
    for k, qr in enumerate(w.queries):
        c, _ = oracle.match(w.graph, qr, rows=False, threads=THREADS, root=BATCH_SLICE)
        lines.append("%d %d" % (k, c))
    write("batch_slice_counts.txt", [
        "Oracle embedding counts of the 512 batching queries (workloads.batch()) on the root slice",
        "query vertex %d, splitmix64(f(v)) %% %d == %d.  Written by make_slice_counts.py (%.0f s)."
        % (BATCH_SLICE[0], BATCH_SLICE[1], BATCH_SLICE[2], time.time() - t),
        "fingerprint %s" % fingerprint(w.graph, w.queries),
        "columns: query index, count"], lines)


def make_serving():
    w = W.serving(nq=SERVING_ARRIVALS)
    t = time.time()
    lines = []
    for k, qr in enumerate(w.queries):
        c, _ = oracle.match(w.graph, qr, rows=False, threads=THREADS, root=(0, SERVING_MOD, k % SERVING_MOD))
        lines.append("%d %d %d" % (k, k % SERVING_MOD, c))
    write("serving_slice_counts.txt", [
        "Oracle embedding counts of the %d arrivals of workloads.serving(nq=%d); arrival k is counted"
        % (SERVING_ARRIVALS, SERVING_ARRIVALS),
        "on the root slice query vertex 0, splitmix64(f(v)) %% %d == k %% %d.  Written by make_slice_counts.py (%.0f s)."
        % (SERVING_MOD, SERVING_MOD, time.time() - t),
        "fingerprint %s" % fingerprint(w.graph, w.queries),
        "columns: arrival index, residue, count"], lines)


# Per shape: the root vertices of a chosen residue all have dmin..dmax
# neighbours, none of degree above maxnd.  With the oracle's order (breadth
# first from query vertex 0) its search from such a root v costs about
#   K4:          deg(v)^3 (the other three vertices are neighbours of v);
#   house+tail:  deg(v)^3 times two neighbour degrees;
#   C5:          (sum of v's neighbour degrees)^2;
# so these bounds keep every slice to seconds while the GPU's slice is the
# same set of embeddings.
LARGE_CRITERIA = {"C5": (3, 12, 1500), "house_tail": (4, 10, 60000), "K4": (16, 64, 1 << 30)}


def residues_by_root_degree(g, dmin, dmax, maxnd_max):
    """Residues r of LARGE_MOD (ascending) whose root vertices (every v with
    hash % mod == r) all meet the degree bounds."""
    d = np.diff(g.row_ptr)
    h = slice_hash_all(g.n) % np.uint64(LARGE_MOD)
    src = np.repeat(np.arange(g.n), d)
    maxnd = np.zeros(g.n, np.int64)
    np.maximum.at(maxnd, src, d[g.col])
    ok = (d >= dmin) & (d <= dmax) & (maxnd <= maxnd_max)
    order = np.argsort(h, kind="stable")
    hs = h[order]
    keys = np.arange(LARGE_MOD, dtype=np.uint64)
    starts, ends = np.searchsorted(hs, keys), np.searchsorted(hs, keys, side="right")
    for r in range(1, LARGE_MOD):
        mem = order[starts[r]:ends[r]]
        if mem.size and ok[mem].all():
            yield r


def make_large():
    g = W.large_graph()
    t = time.time()
    lines = []
    queries = [W.shape(s) for s in LARGE_SHAPES]
    for name, qr in zip(LARGE_SHAPES, queries):
        found = 0
        for tried, r in enumerate(residues_by_root_degree(g, *LARGE_CRITERIA[name])):
            c, _ = oracle.match(g, qr, rows=False, threads=THREADS, root=(0, LARGE_MOD, r))
            if c == 0 and tried < 400:
                continue  # keep slices with embeddings
            lines.append("%s %d %d" % (name, r, c))
            found += 1
            if found == LARGE_RESIDUES:
                break
    write("large_slice_counts.txt", [
        "Oracle embedding counts on the 2^21-vertex unlabelled R-MAT graph (workloads.large_graph()) on",
        "root slices query vertex 0, splitmix64(f(v)) %% %d == r, for residues r whose root vertices" % LARGE_MOD,
        "have few neighbours, of bounded degree (per shape: %s as (min, max degree, max" % LARGE_CRITERIA,
        "neighbour degree)), so the oracle's search from them is small; residues with no embedding are",
        "skipped.  Shapes: workloads.shape().  Written by make_slice_counts.py (%.0f s)." % (time.time() - t),
        "fingerprint %s" % fingerprint(g, queries),
        "columns: shape, residue, count"], lines)


if __name__ == "__main__":
    which = sys.argv[1:] or ["batch", "serving", "large"]
    for name in which:
        {"batch": make_batch, "serving": make_serving, "large": make_large}[name]()
