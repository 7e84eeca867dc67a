"""bench.py's host-side contract: one GPU only (a clear message and exit
code 2 for more, before anything touches a GPU), the per-kernel algorithmic
byte model, and the traffic file lookup (null once the kernel sources
differ from the ones the counters were taken at)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes():
    # the step: codes 1 + A 4 (forward), codes 1 + g 4 + lambda 4 (adjoint)
    assert bench.STEP_BYTES_PER_CELL == 14
    assert bench.KERNEL_BYTES_PER_CELL["adj_pass1"] == 5.0
    assert bench.KERNEL_BYTES_PER_CELL["d8_directions"] == 5.0


def test_traffic_lookup(tmp_path, monkeypatch):
    sha = bench.source_sha()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_sha", lambda: sha)
    (tmp_path / "profiles").mkdir()
    assert bench.measured_traffic("adj_pass1", "dem32768_64x32") is None       # no file
    f = tmp_path / "profiles" / "traffic_adj_pass1_dem32768_64x32.txt"
    f.write_text(f"# test\nsource_sha = {sha}\ntraffic_bytes_per_launch = 123\n")
    assert bench.measured_traffic("adj_pass1", "dem32768_64x32") == 123.0
    f.write_text("source_sha = 0000000000000000\ntraffic_bytes_per_launch = 123\n")
    assert bench.measured_traffic("adj_pass1", "dem32768_64x32") is None       # stale counters

