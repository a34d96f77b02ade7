"""Whole-chain sweeps (MC_WHOLE_CHAINS: one lane per chain, a single exact
scan from the chain start) against the FP64 reference: splitting iterates
after 1, 3 and 20 iterations, exact cuts against max-flow, and the
alpha-expansion moves, whose flat chains are what the option is for."""
import numpy as np
import pytest

import oracle
from oracle import multilabel as ml
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


@pytest.mark.parametrize("shape,variant", [((37, 53), 1), ((37, 53), 2), ((6, 17, 23), 2), ((1, 70), 1),
                                           ((70, 1), 1)])
@pytest.mark.parametrize("iters", [1, 3, 20])
def test_iterates_match_reference(dev, shape, variant, iters):
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 900 + iters)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=iters, gap_tol=0.0, variant=variant,
                      whole_chains=True)
    ref = oracle.dr_solve(w, a, variant=variant - 1, max_iters=iters, gap_tol=0.0)
    x = res.x.cpu().numpy()
    scale = max(1.0, np.abs(ref["x"]).max())
    assert np.abs(x - ref["x"]).max() / scale <= REL_TOL


@pytest.mark.parametrize("shape", [(3, 4000), (4000, 2), (2, 3071), (2, 3072)])
@pytest.mark.parametrize("iters", [2, 9])
def test_long_chains_match_reference(dev, shape, iters):
    """Chains too long to stage whole in LDS (more than 3071 positions) are
    read from global memory; both kinds, and the boundary, against the
    reference iterates."""
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 950 + iters)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=iters, gap_tol=0.0, whole_chains=True)
    ref = oracle.dr_solve(w, a, max_iters=iters, gap_tol=0.0)
    x = res.x.cpu().numpy()
    scale = max(1.0, np.abs(ref["x"]).max())
    assert np.abs(x - ref["x"]).max() / scale <= REL_TOL


@pytest.mark.parametrize("shape,variant", [((16320, 4), 1), ((16321, 4), 1), ((16384, 4), 1),
                                           ((4, 128, 130), 2), ((4, 120, 136), 2)])
@pytest.mark.parametrize("iters", [2, 7])
def test_many_chains_take_the_global_sweep(dev, shape, variant, iters):
    """Families of 16321 chains or more (256 or more 64-chain waves) take the
    global-memory whole-chain sweep over many blocks, fewer the LDS one: the
    2D boundary 16320 / 16321 rows, 16384 rows, and volumes whose depth
    family has 16640 (global) and 16320 (LDS) chains, in the product space;
    iterates against the reference, then the exact cut against max-flow."""
    from paper_1503_01563_amd import mc
    w, a = gen.iid_grid(shape, 970 + iters)
    wt, at = T(w, dev), [T(x, dev) for x in a]
    res = mc.tv_solve(wt, at, max_iters=iters, gap_tol=0.0, variant=variant, whole_chains=True)
    ref = oracle.dr_solve(w, a, variant=variant - 1, max_iters=iters, gap_tol=0.0)
    x = res.x.cpu().numpy()
    scale = max(1.0, np.abs(ref["x"]).max())
    assert np.abs(x - ref["x"]).max() / scale <= REL_TOL
    if iters == 7:
        res = mc.tv_solve(wt, at, max_iters=3000, check_every=2, variant=variant, whole_chains=True)
        assert res.converged and res.energy == oracle.mincut(w, a, "dinic")[0]


@pytest.mark.parametrize("seed", range(1000, 1006))
def test_exact_against_maxflow(dev, seed):
    from paper_1503_01563_amd import mc
    w, a = gen.config_small(seed)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=2000, check_every=2, whole_chains=True)
    assert res.converged
    assert res.energy == oracle.mincut(w, a, "dinic")[0]


def test_volume_and_image_exact(dev):
    from paper_1503_01563_amd import mc
    w, a = gen.ellipse_grid((12, 40, 56), 3100, lam=1.5)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4, whole_chains=True)
    assert res.converged and res.energy == oracle.mincut(w, a, "dinic")[0]
    w, a = gen.config_image2d(2001, (256, 256))
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4, whole_chains=True)
    assert res.converged and res.energy == oracle.mincut(w, a, "dinic")[0]


def test_alpha_expansion_with_whole_chains(dev):
    import torch
    from paper_1503_01563_amd import mc
    data, lam, _ = gen.stereo_labels((96, 128), 6800, n_labels=10)
    labels = torch.zeros((96, 128), dtype=torch.int32, device=dev)
    res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 1, 2.0, whole_chains=True)
    assert res.converged and res.uncertified == 0
    f = labels.cpu().numpy()
    assert res.energy == ml.energy(data, lam, 1, 2.0, f)
    for alpha in range(10):
        w, a = ml.expansion_problem(data, lam, 1, 2.0, f, alpha)
        assert oracle.mincut(w, a)[0] >= 0


def test_automatic_choice(dev):
    """With neither kind forced the solver sweeps whole chains on flat move
    problems and keeps pieces on noisy grids; both stay exact."""
    from paper_1503_01563_amd import mc
    data, lam, _ = gen.stereo_labels((96, 128), 6900, n_labels=8)
    w, a = ml.expansion_problem(data, lam, 1, 2.0, np.zeros((96, 128), np.int64), 1)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4)
    assert res.converged and res.whole_chains == 1
    assert res.energy == oracle.mincut(w, a)[0]
    w, a = gen.config_image2d(2002, (256, 256))
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4)
    assert res.converged and res.whole_chains == 0
    assert res.energy == oracle.mincut(w, a, "dinic")[0]
    forced = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4, whole_chains=True)
    assert forced.whole_chains == 1 and forced.energy == res.energy
    pieces = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=3000, check_every=4, whole_chains=False)
    assert pieces.whole_chains == 0 and pieces.energy == res.energy


@pytest.mark.parametrize("variant", ["bcd", "ap", "fista"])
def test_other_outer_iterations_with_whole_chains(dev, variant):
    from paper_1503_01563_amd import mc
    var = {"bcd": mc.VARIANT_BCD, "ap": mc.VARIANT_AP, "fista": mc.VARIANT_FISTA}[variant]
    w, a = gen.iid_grid((40, 48), 5100)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=20000, check_every=2, variant=var,
                      whole_chains=True)
    assert res.converged and res.whole_chains == 1
    assert res.energy == oracle.mincut(w, a, "dinic")[0]


def test_grid8_with_whole_chains(dev):
    from oracle import grid8 as G8
    from paper_1503_01563_amd import mc
    w, a = gen.ellipse_grid8((64, 80), 5200)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=5000, check_every=2, whole_chains=True)
    assert res.converged
    assert res.energy == G8.mincut(w, a)[0]


@pytest.mark.parametrize("variant", ["bcd", "fista", "bcd_dr"])
def test_automatic_choice_in_other_solvers(dev, variant):
    from paper_1503_01563_amd import mc
    var = {"bcd": mc.VARIANT_BCD, "fista": mc.VARIANT_FISTA, "bcd_dr": mc.VARIANT_BCD_DR}[variant]
    data, lam, _ = gen.stereo_labels((96, 128), 6900, n_labels=8)
    w, a = ml.expansion_problem(data, lam, 1, 2.0, np.zeros((96, 128), np.int64), 1)
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=20000, check_every=2, variant=var)
    assert res.converged and res.whole_chains == 1
    assert res.energy == oracle.mincut(w, a)[0]
    w, a = gen.config_image2d(2002, (256, 256))
    res = mc.tv_solve(T(w, dev), [T(x, dev) for x in a], max_iters=20000, check_every=2, variant=var)
    assert res.converged and res.whole_chains == 0
    assert res.energy == oracle.mincut(w, a, "dinic")[0]
