"""Host-side checks of the C-ABI library (no GPU needed): it builds, loads and
exports every function include/mc.h declares, and the header's structs match
the binding's ctypes layouts."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1503_01563_amd import mc
    if not os.path.exists(mc.LIB_PATH):
        from paper_1503_01563_amd import build
        build.build()
    return mc.LIB_PATH


def test_header_declares_boundary():
    names = declared_functions()
    for n in ("mc_tv_solve", "mc_tv_prox_chains", "mc_cut_energy", "mc_tv_solve_batched", "mc_ctx_create",
              "mc_ctx_destroy", "mc_status_string", "mc_last_error", "mc_opts_default", "mc_ws_param_count",
              "mc_ws_forward", "mc_ws_backward", "mc_ws_adam_step", "mc_ws_warm_state",
              "mc_expansion_problem", "mc_ml_energy", "mc_alpha_expansion"):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(libpath)
    for n in declared_functions():
        assert hasattr(lib, n)


def test_host_only_calls(libpath):
    from paper_1503_01563_amd import mc
    lib = mc.load_library()
    o = mc.Opts()
    lib.mc_opts_default(ctypes.byref(o))
    assert o.max_iters == 500 and o.check_every == 1 and abs(o.gap_tol - 1e-3) < 1e-15
    assert abs(o.tau0 - 1e-3) < 1e-9 and o.variant == 0
    assert lib.mc_status_string(0) == b"ok"
    assert b"converged" in lib.mc_status_string(1)
    # null context is rejected without touching a device
    assert lib.mc_tv_prox_chains(None, None, 0, None, None, None, None, None) == -1
    assert b"ctx" in lib.mc_last_error()
    assert lib.mc_ctx_destroy(None) == 0
    # warm-start network: parameter count agrees with the reference layout
    from oracle import convnet
    assert mc.ws_param_count() == convnet.param_count() == 19970
    assert lib.mc_ws_forward(None, None, 1, 1, 1, None, None, None, None, None) == -1
    assert lib.mc_ws_adam_step(None, None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-8, None) == -1
    assert lib.mc_ws_warm_state(None, None, None, None, 0.0, None, None) == -1
    # alpha-expansion entry points reject a null context before any device work
    assert lib.mc_expansion_problem(None, None, 2, None, None, 0, 0.0, None, 0, None, None, None) == -1
    assert lib.mc_ml_energy(None, None, 2, None, None, 0, 0.0, None, None, None) == -1
    assert lib.mc_alpha_expansion(None, None, 2, None, None, 0, 0.0, None, 1, None, None, None) == -1


def test_struct_layouts_match_header():
    from paper_1503_01563_amd import mc
    assert ctypes.sizeof(mc.Grid) == 32
    assert ctypes.sizeof(mc.Opts) == 48
    assert ctypes.sizeof(mc.Stats) == 88
    assert mc.Stats.ms.offset == 44 and mc.Opts.flags.offset == 24
    assert mc.Stats.dual_sweep_ms.offset == 72 and mc.Stats.dual_sweep_launches.offset == 80
    assert mc.Opts.batch_items.offset == 28 and mc.Opts.bcd_iters.offset == 32 and mc.Opts.reserved.offset == 36
    assert ctypes.sizeof(mc.MLStats) == 56
    assert (mc.MLStats.dr_iters.offset, mc.MLStats.energy0.offset, mc.MLStats.energy.offset,
            mc.MLStats.ms.offset) == (24, 32, 40, 48)
