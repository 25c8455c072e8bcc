"""bench.py's contract pieces that need no GPU."""
import json
import os
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_fused_bytes_per_point():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.fused_bytes(3, 8) == 816
    assert bench.fused_bytes(3, 4) == 408
    assert bench.fused_bytes(1, 8) == 144
    assert bench.fused_bytes(2, 8) == 392


def test_traffic_record_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = {"kernel_hash": bench.kernel_hash(), "n": 1 << 24, "bytes_per_launch": 1.0}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(p))
    assert bench.measured_traffic(1 << 24) == 1.0
    assert bench.measured_traffic(1 << 20) is None
    rec["kernel_hash"] = "stale"
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(1 << 24) is None
