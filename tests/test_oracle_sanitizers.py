"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a C driver calls every exported function on small seeded
inputs and edge cases; any out-of-bounds access, leak or undefined behaviour
aborts the run.  Also checks that the OpenMP build of the same source gives
bit-identical results to the plain one."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from tests.conftest import ROOT


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "orc_asan")
    src = [os.path.join(ROOT, "tests", "oracle_asan_driver.c"), os.path.join(ROOT, "oracle", "oracle.c")]
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-Wno-unknown-pragmas", "-o", exe] + src + ["-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failed checks" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_openmp_build_is_bit_identical():
    from paper_1503_01563_amd import gen
    oracle.build(force=False)
    for w, a, kw in ((*gen.ellipse_grid((96, 128), 2301), {}), (*gen.iid_grid((64, 64), 1001), {}),
                     (*gen.ellipse_grid((12, 20, 24), 3301, lam=1.5), {})):
        r1 = oracle.dr_solve(w, a, max_iters=40, gap_tol=0, return_z=True, **kw)
        r4 = oracle.dr_solve(w, a, max_iters=40, gap_tol=0, return_z=True, threads=4, **kw)
        for k in ("x", "labels", "z"):
            assert np.array_equal(r1[k], r4[k]), k
        for k in ("cert", "energy", "lower_bound", "tv_gap", "tau_used", "iters"):
            assert r1[k] == r4[k], k
