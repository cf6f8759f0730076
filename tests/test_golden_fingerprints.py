"""The stored oracle counts (tests/golden/*_slice_counts.txt) were taken on the
workloads the generators produce now: their fingerprints match."""
import pytest

from paper_2003_01527_amd import workloads as W

from golden.make_slice_counts import SERVING_ARRIVALS, fingerprint
from golden_io import GOLDEN


def stored(fname):
    for line in open(GOLDEN + "/" + fname):
        if line.startswith("# fingerprint"):
            return line.split()[2]
    raise AssertionError("no fingerprint in " + fname)


def test_batch_fingerprint():
    w = W.batch()
    assert fingerprint(w.graph, w.queries) == stored("batch_slice_counts.txt")


def test_serving_fingerprint():
    w = W.serving(nq=SERVING_ARRIVALS)
    assert fingerprint(w.graph, w.queries) == stored("serving_slice_counts.txt")


@pytest.mark.slow
def test_large_fingerprint():
    shapes = []
    for line in open(GOLDEN + "/large_slice_counts.txt"):
        if not line.startswith("#") and line.split()[0] not in shapes:
            shapes.append(line.split()[0])
    assert fingerprint(W.large_graph(), [W.shape(s) for s in shapes]) == stored("large_slice_counts.txt")
