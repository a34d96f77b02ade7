"""Sweeps of volumes in long pieces streamed through an LDS ring: the same
iterates as the short pieces, bit for bit on the bench volume (both are the
exact scan from a knot of the true solution or the chain start), and the
same certificate; to FP32 rounding on odd-sized volumes with short segments,
long constant segments (lanes that fall behind the ring, positions evicted
before they are final) and one segment per chain, where the primal built
from the streamed dual sweep's edge duals is compared too."""
import numpy as np
import pytest

import oracle
from paper_1503_01563_amd import gen

pytestmark = pytest.mark.gpu
REL_TOL = 1e-4


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1503_01563_amd import mc
    mc.load_library()
    return torch.device("cuda:0")


def T(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("iters", [3, 9])
def test_streamed_sweeps_equal_piece_sweeps(dev, iters):
    """256x256x128: 3072 waves of streamed pieces after the first sweep;
    MC_PIECE_CHAINS keeps the short pieces.  Same state bit for bit."""
    from paper_1503_01563_amd import mc
    w, a = gen.config_volume3d(3000)
    wt, at = T(w, dev), [T(x, dev) for x in a]
    ref = mc.tv_solve(wt, at, max_iters=iters, check_every=4, gap_tol=0.0, return_z=True, whole_chains=False)
    res = mc.tv_solve(wt, at, max_iters=iters, check_every=4, gap_tol=0.0, return_z=True)
    assert res.whole_chains == 0 and ref.whole_chains == 0
    assert bool((res.z == ref.z).all()), float((res.z - ref.z).abs().max())
    assert res.energy == ref.energy
    assert abs(res.cert_gap - ref.cert_gap) <= 1e-6 * max(1.0, abs(ref.lower_bound))


@pytest.mark.parametrize("shape,case", [((160, 200, 300), "iid"), ((160, 200, 300), "smooth"),
                                        ((160, 200, 300), "flat"), ((40, 300, 1000), "smooth")])
def test_streamed_volumes_match_piece_sweeps(dev, shape, case):
    """160x200x300 (D x H x W): rows in two pieces of 150, columns in two of
    100, depth chains whole (160), ragged last chain groups; 40x300x1000:
    rows in eight pieces of 125, depth chains of 40.  Short segments (iid
    integers), long constant ones (a strongly smoothed image) and chains of
    one segment each (a constant input).  Against the short pieces to FP32
    rounding: with exact ties (integer data) two exact scans may split a
    constant run into segments differently, and round differently."""
    from paper_1503_01563_amd import mc
    if case == "iid":
        w, a = gen.iid_grid(shape, 995)
    elif case == "smooth":
        w, a = gen.ellipse_grid(shape, 996, lam=6.0)
    else:
        w = np.full(shape, 0.75, np.float32)
        _, a = gen.ellipse_grid(shape, 997, lam=1.0)
    wt, at = T(w, dev), [T(x, dev) for x in a]
    ref = mc.tv_solve(wt, at, max_iters=7, check_every=4, gap_tol=0.0, return_x=True, return_z=True,
                      whole_chains=False)
    res = mc.tv_solve(wt, at, max_iters=7, check_every=4, gap_tol=0.0, return_x=True, return_z=True)
    scale = max(1.0, float(ref.z.abs().max()))
    assert float((res.z - ref.z).abs().max()) / scale <= 1e-5
    # x is built from the edge duals of the last (streamed, dual) sweep
    xs = max(1.0, float(ref.x.abs().max()))
    assert float((res.x - ref.x).abs().max()) / xs <= 1e-5


def test_streamed_volume_matches_reference(dev):
    """The bench volume after 5 iterations (3 of them streamed) against the
    FP64 reference iteration."""
    from paper_1503_01563_amd import mc
    w, a = gen.config_volume3d(3000)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=5, check_every=5, gap_tol=0.0, return_x=True,
                      return_z=True)
    ref = oracle.dr_solve(w, a, variant=1, max_iters=5, gap_tol=0.0, return_z=True, threads=16)
    x = res.x.cpu().numpy()
    assert np.abs(x - ref["x"]).max() / max(1.0, np.abs(ref["x"]).max()) <= REL_TOL
    z = res.z.cpu().numpy().ravel()
    assert np.abs(z - ref["z"]).max() / max(1.0, np.abs(ref["z"]).max()) <= REL_TOL


@pytest.mark.parametrize("shape", [(12, 40, 56), (96, 80)])
def test_dual_sweep_time_is_reported(dev, shape):
    """MC_PROFILE: the sweep time of the launches that also wrote edge duals
    (the certificate iterations) is reported apart; their number follows the
    check schedule (one launch per iteration in the product space, two in
    the two-set form)."""
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 1234)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=9, check_every=4, gap_tol=0.0, profile=True)
    per_it = 1 if len(shape) == 3 else 2
    assert res.checks == 3
    assert res.dual_sweep_launches == 3 * per_it
    assert 0.0 < res.dual_sweep_ms < res.sweep_ms
