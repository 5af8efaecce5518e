"""Host-side parts of the benchmark's output contract (no GPU needed)."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def _sources_hash():
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def test_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    prof = tmp_path / "counters.txt"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.measured_traffic() is None            # no summary
    prof.write_text(f"traffic_bytes_per_launch: 1234567\nkernel_sources_sha256: {_sources_hash()}\n")
    assert bench.measured_traffic() == 1234567.0
    prof.write_text("traffic_bytes_per_launch: 1234567\nkernel_sources_sha256: " + "0" * 64 + "\n")
    assert bench.measured_traffic() is None            # kernel changed since the counters were taken
