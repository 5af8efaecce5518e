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


def test_valu_busy_only_for_the_profiled_sources(tmp_path, monkeypatch):
    prof = tmp_path / "sq.txt"
    monkeypatch.setattr(bench, "SQ_PROFILE", str(prof))
    assert bench.measured_valu_busy() is None
    body = ("valu_issue_share: 0.8\nvector_instructions_per_wave_event: 250\nscalar_instructions_per_wave_event: 130\n")
    prof.write_text(body + f"kernel_sources_sha256: {_sources_hash()}\n")
    assert bench.measured_valu_busy()["valu_issue_share"] == 0.8
    prof.write_text(body + "kernel_sources_sha256: " + "0" * 64 + "\n")
    assert bench.measured_valu_busy() is None


def test_work_count_per_event():
    """The per-part algorithmic count of one direct-method step."""
    from paper_0912_2551_amd import workloads as W
    assert bench.n_predicates(W.C2_FORMULA) == 3 and bench.n_predicates(W.C1_FORMULA) == 1
    assert bench.work_slots_per_event(W.michaelis_menten(), 3) == 192
    assert bench.work_slots_per_event(W.immigration_death(), 1) == 181
    net = W.c3_network()
    assert bench.n_predicates(W.c3_formula(net)) == 4
    assert bench.work_slots_per_event(net, 4) == 1228
