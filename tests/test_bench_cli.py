"""bench.py's command line without a GPU: more than one GPU is refused with a
message and exit status 2, before any device is touched."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_needs_matching_sources_and_vertex_order(tmp_path, monkeypatch):
    # a stored HBM-traffic record is reported only for the sources and the
    # vertex order it was measured on
    import json
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench
    rec = {"sources_sha1": bench.sources_sha1(), "vertex_order": "degree", "traffic_bytes_per_launch": 123}
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "traffic_record_path", lambda workload: str(path))
    assert bench.measured_traffic("large", "degree") == 123
    assert bench.measured_traffic("large", "caller") is None
    rec["sources_sha1"] = "0" * 40
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("large", "degree") is None
    monkeypatch.setattr(bench, "traffic_record_path", lambda workload: str(tmp_path / "missing.json"))
    assert bench.measured_traffic("large", "degree") is None
