"""Identical inputs give identical outputs: every reduction has a fixed order
and no floating-point atomics are used, so repeated solves agree bit for bit
(primal, labels, statistics)."""
import numpy as np
import pytest

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


def T(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("case", ["image2d", "volume3d", "whole_chains"])
def test_repeated_solves_are_bitwise_identical(dev, case):
    from paper_1503_01563_amd import mc
    if case == "volume3d":
        w, a = gen.ellipse_grid((24, 48, 64), 3300, lam=1.5)
    else:
        w, a = gen.config_image2d(2004, (320, 384))
    kw = {"whole_chains": True} if case == "whole_chains" else {}
    runs = [mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4, **kw) for _ in range(3)]
    for r in runs[1:]:
        assert np.array_equal(r.x.cpu().numpy().view(np.uint32), runs[0].x.cpu().numpy().view(np.uint32))
        assert np.array_equal(r.labels.cpu().numpy(), runs[0].labels.cpu().numpy())
        assert (r.iters, r.energy, r.cert_gap, r.lower_bound, r.tv_gap) == \
            (runs[0].iters, runs[0].energy, runs[0].cert_gap, runs[0].lower_bound, runs[0].tv_gap)


def test_repeated_alpha_expansion_is_identical(dev):
    import torch
    from paper_1503_01563_amd import mc
    data, lam, _ = gen.stereo_labels((80, 96), 6950, n_labels=8)
    outs = []
    for _ in range(2):
        labels = torch.zeros((80, 96), dtype=torch.int32, device=dev)
        res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 1, 2.0)
        outs.append((labels.cpu().numpy(), res.energy, res.dr_iters, res.accepted))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]


@pytest.mark.parametrize("case,check_every,max_iters", [
    ("image2d", 4, 3000), ("image2d", 3, 3000), ("image2d", 1, 3000), ("image2d", 2, 15),
    ("product2d", 4, 3000), ("volume3d", 4, 3000), ("volume3d", 2, 11), ("warm2d", 2, 3000)])
def test_overlapped_checks_match_checks_read_at_once(dev, case, check_every, max_iters):
    """From a solve's third check on, a check is read while the next
    iteration already runs (the default); with MC_PROFILE every check is read
    at once.  Both end on the same certified iteration with the same primal,
    labels, state and statistics, also when max_iters stops the solve."""
    from paper_1503_01563_amd import mc
    if case == "volume3d":
        w, a = gen.ellipse_grid((24, 48, 64), 3301, lam=1.5)
    else:
        w, a = gen.config_image2d(2005, (256, 320))
    kw = {"variant": mc.VARIANT_PRODUCT} if case == "product2d" else {}
    wt, at = T(w, dev), [T(x, dev) for x in a]
    if case == "warm2d":
        kw["z0"] = mc.tv_solve(wt, at, max_iters=12, check_every=12, gap_tol=0.0, return_z=True).z
    runs = [mc.tv_solve(wt, at, max_iters=max_iters, check_every=check_every, return_z=True, profile=prof, **kw)
            for prof in (False, True)]
    r, ref = runs
    assert ref.converged or max_iters < 3000
    assert (r.iters, r.converged, r.checks, r.energy, r.cert_gap, r.lower_bound, r.tv_gap) == \
        (ref.iters, ref.converged, ref.checks, ref.energy, ref.cert_gap, ref.lower_bound, ref.tv_gap)
    assert np.array_equal(r.x.cpu().numpy().view(np.uint32), ref.x.cpu().numpy().view(np.uint32))
    assert np.array_equal(r.labels.cpu().numpy(), ref.labels.cpu().numpy())
    assert np.array_equal(r.z.cpu().numpy().view(np.uint32), ref.z.cpu().numpy().view(np.uint32))
    assert r.ms > 0


@pytest.mark.parametrize("check_every,max_iters", [(4, 3000), (3, 11)])
def test_overlapped_checks_match_8connected(dev, check_every, max_iters):
    from paper_1503_01563_amd import mc
    w, a = gen.ellipse_grid8((96, 128), 3302)
    wt, at = T(w, dev), [T(x, dev) for x in a]
    r, ref = [mc.tv_solve(wt, at, max_iters=max_iters, check_every=check_every, return_z=True, profile=prof)
              for prof in (False, True)]
    assert ref.converged or max_iters < 3000
    assert (r.iters, r.converged, r.checks, r.energy, r.cert_gap, r.lower_bound) == \
        (ref.iters, ref.converged, ref.checks, ref.energy, ref.cert_gap, ref.lower_bound)
    assert np.array_equal(r.x.cpu().numpy().view(np.uint32), ref.x.cpu().numpy().view(np.uint32))
    assert np.array_equal(r.labels.cpu().numpy(), ref.labels.cpu().numpy())
    assert np.array_equal(r.z.cpu().numpy().view(np.uint32), ref.z.cpu().numpy().view(np.uint32))
