"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def parse_edges(tokens):
    return [tuple(int(x) for x in t.split("-")) for t in tokens]


def automorphisms():
    out = []
    for line in open(os.path.join(GOLDEN, "automorphisms.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        out.append((tok[0], int(tok[1]), parse_edges(tok[2:])))
    return out


def records(fname):
    """Blocks of 'key values...' lines separated by comment lines starting '#'."""
    blocks, cur = [], {}
    for line in open(os.path.join(GOLDEN, fname)):
        s = line.strip()
        if not s:
            continue
        if s.startswith("#"):
            if cur:
                blocks.append(cur)
                cur = {}
            continue
        tok = s.split()
        cur[tok[0]] = tok[1:]
    if cur:
        blocks.append(cur)
    return blocks


def ints(tok):
    return None if tok == ["-"] else [int(x) for x in tok]


def query_of(edges, labels=None, name=""):
    from paper_2003_01527_amd.workloads import Query
    e = np.array(edges, dtype=np.int32).reshape(-1, 2)
    q = 1 + int(e.max())
    return Query(q, e, None if labels is None else np.array(labels, np.int32), None, -1.0, name)
