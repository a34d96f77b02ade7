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
    assert a.seed == 3000 and a.size == 1024 and a.image_seed == 2000 and not a.cpu_full


@pytest.mark.parametrize("path,voxels,bytes_per_voxel", [
    (bench.TRAFFIC_PROFILE, 256 * 256 * 128, bench.VOL_BYTES_VALUE),
    (bench.IMG_TRAFFIC_PROFILE, 1024 * 1024, bench.IMG_BYTES_PER_VOXEL_SWEEP)])
def test_traffic_summary_is_readable(path, voxels, bytes_per_voxel):
    """The committed counter summaries carry the two lines the benchmark reads;
    a figure is reported only while the sweep sources match its hash."""
    text = open(path).read()
    h = re.search(r"sweep sources sha256\[:16\]: `([0-9a-f]+)`", text)
    v = re.search(r"HBM bytes per sweep launch: `([0-9.eE+]+)`", text)
    assert h and v
    t = bench.measured_traffic(path)
    if h.group(1) == bench.sweep_sources_hash():
        assert t == float(v.group(1))
        # counted bytes cannot be below the algorithmic bytes of a launch by
        # more than the counters' granularity
        assert t > 0.9 * bytes_per_voxel * voxels
    else:
        assert t is None


def test_cpu_threads_follow_the_host_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.cpu_threads() == 3
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.cpu_threads() >= 1


@pytest.mark.parametrize("name", ["volume3d_256x256x128_solve_kernel_stats.md",
                                  "volume3d_256x256x128_sweep_traffic.md",
                                  "image2d_1024_sweep_traffic.md"])
def test_profiles_name_their_command(name):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    assert "rocprofv3" in text and "bench.py" in text
