"""Reusing one frame's dual in the next (the paper's warm start across related
problems): every frame of a drifting-ellipse sequence is still solved exactly
(energy equal to max-flow), with fewer iterations than from a cold start."""
import numpy as np
import pytest

import oracle
from paper_1503_01563_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_01563_amd import mc
    mc.load_library()
    return torch.device("cuda:0")


def test_dual_reuse_state_is_feasible_for_new_weights(dev):
    import torch
    from paper_1503_01563_amd import mc, warmstart
    frames = gen.ellipse_sequence((40, 56), 5100, 2)
    (w0, a0), (w1, a1) = frames
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
    r = mc.tv_solve(T(w0), [T(a0[0]), T(a0[1])], max_iters=50, gap_tol=0.0, return_z=True)
    z0 = warmstart.dual_reuse_state(r.z, T(a0[0]), None, T(a1[0]), c=0.0)
    # with c = 0 the state is D^T p with |p| <= a_new: its row prox is zero
    q = mc.tv_prox_chains(z0, T(a1[0]), 0).cpu().numpy()
    assert np.abs(q).max() < 1e-3


def _check_exact(rows, frames):
    for r, (w, a) in zip(rows, frames):
        e_star = oracle.mincut(w, a, "dinic")[0]
        assert r["cold_ok"] and r["warm_ok"], r
        assert r["cold_energy"] == e_star and r["warm_energy"] == e_star, r


def _totals(rows):
    return (sum(r["cold_iters"] for r in rows[1:]), sum(r["warm_iters"] for r in rows[1:]),
            sum(r["cold_ms"] for r in rows[1:]), sum(r["warm_ms"] for r in rows[1:]))


def test_edit_sequence_dual_reuse_exact_and_faster(dev):
    """Integer grid with 2 % of the unaries redrawn per frame: reusing the
    previous frame's dual cuts the iterations; every frame stays exact."""
    from paper_1503_01563_amd import warmstart
    frames = gen.edit_sequence((256, 256), 7000, 8, frac=0.02)
    rows = warmstart.sequence_compare(frames)
    _check_exact(rows, frames)
    cold, warm, cms, wms = _totals(rows)
    print("edits, frames 1..7: iterations cold %d warm %d; ms cold %.1f warm %.1f" % (cold, warm, cms, wms))
    assert warm < cold


def test_video_sequence_dual_reuse_exact(dev):
    """Drifting ellipses with fresh noise per frame: cold starts already
    certify within a few tens of iterations; reuse must stay exact."""
    from paper_1503_01563_amd import warmstart
    frames = gen.ellipse_sequence((256, 256), 5000, 8)
    rows = warmstart.sequence_compare(frames)
    _check_exact(rows, frames)
    cold, warm, cms, wms = _totals(rows)
    print("video, frames 1..7: iterations cold %d warm %d; ms cold %.1f warm %.1f" % (cold, warm, cms, wms))
