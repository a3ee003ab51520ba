"""Host logic of bench.py that needs no GPU: the one-GPU refusal and the
counter summary's source check."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    c = json.load(open(bench.COUNTERS_FILE))
    if c["kernel_source_sha"] == bench.source_digest():
        assert bench.hbm_traffic(1) == c["hbm_bytes_per_launch"]
    else:
        assert bench.hbm_traffic(1) is None
    stale = dict(c, kernel_source_sha="0" * 16)
    f = tmp_path / "c.json"
    f.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    assert bench.hbm_traffic(1) is None
