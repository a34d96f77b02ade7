"""The benchmark's command-line contract, checked without a GPU: one JSON
line per run on one GPU, a clear refusal of multi-GPU runs, and a counter
summary whose format the benchmark can read."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_multi_gpu_runs_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_defaults_are_one_gpu_and_a_short_run(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.steps == 5 and a.warmup == 1 and a.check_every == 4
    assert a.size == 1024 and a.seed == 2000


def test_traffic_summary_is_readable():
    """The committed counter summary carries the two lines the benchmark reads;
    the figure is reported only while the sweep sources match its hash."""
    text = open(bench.TRAFFIC_PROFILE).read()
    h = re.search(r"sweep sources sha256\[:16\]: `([0-9a-f]+)`", text)
    v = re.search(r"HBM bytes per sweep launch: `([0-9.eE+]+)`", text)
    assert h and v
    t = bench.measured_traffic()
    if h.group(1) == bench.sweep_sources_hash():
        assert t == float(v.group(1))
        # counted bytes cannot be below the algorithmic bytes of a launch by
        # more than the counters' granularity
        assert t > 0.9 * bench.BYTES_PER_VOXEL_SWEEP * 1024 * 1024
    else:
        assert t is None


@pytest.mark.parametrize("name", ["image2d_1024_solve_kernel_stats.md", "image2d_1024_sweep_traffic.md"])
def test_profiles_name_their_command(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert "rocprofv3" in text and "bench.py" in text
