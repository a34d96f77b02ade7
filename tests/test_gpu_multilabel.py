"""GPU alpha-expansion (multi-label energies as a series of exact cuts, Sec.
4.4 and 6.1 of the paper) against the FP64 reference: move problems and
energies element by element, every move's cut exact against max-flow, and the
result a local minimum for every expansion (checked by max-flow).  Moves on
ties may pick different optimal cuts than the reference, so whole runs are
compared by what is unique: the energy of the labels and their optimality
against every expansion."""
import numpy as np
import pytest

import oracle
from oracle import multilabel as ml
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


def Ti(x, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(dev)


def problem(shape, seed, L):
    data, lam, _ = gen.stereo_labels(shape, seed, n_labels=L)
    return data, lam


KINDS = [(0, 0.0), (1, 2.0)]  # (Potts, -), (truncated linear, T = 2)


@pytest.mark.parametrize("shape", [(37, 53), (9, 300), (1, 17), (23, 1)])
@pytest.mark.parametrize("kind,trunc", KINDS)
def test_move_problem_matches_reference(dev, shape, kind, trunc):
    from paper_1503_01563_amd import mc
    L = 6
    data, lam = problem(shape, 6100, L)
    rng = np.random.Generator(np.random.PCG64(17))
    f = rng.integers(0, L, size=shape).astype(np.int32)
    for alpha in range(L):
        w, a = mc.expansion_problem(T(data, dev), [T(x, dev) for x in lam], Ti(f, dev), alpha, kind, trunc)
        rw, ra = ml.expansion_problem(data, lam, kind, trunc, f, alpha)
        assert np.array_equal(w.cpu().numpy().astype(np.float64), rw), alpha
        assert np.array_equal(a[0].cpu().numpy().astype(np.float64), ra[0]), alpha
        assert np.array_equal(a[1].cpu().numpy().astype(np.float64), ra[1]), alpha


@pytest.mark.parametrize("kind,trunc", KINDS)
def test_energy_matches_reference(dev, kind, trunc):
    from paper_1503_01563_amd import mc
    L = 9
    data, lam = problem((41, 67), 6200, L)
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(3):
        f = rng.integers(0, L, size=(41, 67)).astype(np.int32)
        e = mc.ml_energy(T(data, dev), [T(x, dev) for x in lam], Ti(f, dev), kind, trunc)
        assert e == ml.energy(data, lam, kind, trunc, f)


def test_moves_are_exact_cuts(dev):
    """Each move solved by mc_tv_solve reaches the max-flow minimum of its problem."""
    from paper_1503_01563_amd import mc
    L = 8
    data, lam = problem((64, 80), 6300, L)
    f = np.argmin(data, axis=0).astype(np.int32)
    for alpha in range(L):
        w, a = mc.expansion_problem(T(data, dev), [T(x, dev) for x in lam], Ti(f, dev), alpha, 1, 2.0)
        res = mc.tv_solve(w, a, max_iters=5000, check_every=2)
        assert res.converged, alpha
        rw, ra = ml.expansion_problem(data, lam, 1, 2.0, f, alpha)
        e_star = oracle.mincut(rw, ra)[0]
        assert res.energy == e_star, alpha
        assert oracle.cut_energy(rw, ra, res.labels.cpu().numpy()) == e_star


def check_local_optimum(data, lam, kind, trunc, f):
    for alpha in range(data.shape[0]):
        w, a = ml.expansion_problem(data, lam, kind, trunc, f, alpha)
        assert oracle.mincut(w, a)[0] >= 0, alpha


@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("kind,trunc", KINDS)
@pytest.mark.parametrize("shape,L,seed", [((48, 64), 8, 6400), ((33, 75), 5, 6401)])
def test_alpha_expansion_reaches_a_local_minimum(dev, kind, trunc, shape, L, seed, warm):
    from paper_1503_01563_amd import mc
    data, lam = problem(shape, seed, L)
    labels = Ti(np.zeros(shape), dev)
    res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, kind, trunc, warm=warm)
    assert res.converged and res.uncertified == 0
    # every cycle visits every label once: solved or skipped as unchanged
    assert res.moves + res.skipped == res.cycles * L and res.skipped > 0
    f = labels.cpu().numpy()
    assert f.min() >= 0 and f.max() < L
    e = ml.energy(data, lam, kind, trunc, f)
    assert res.energy == e
    assert res.energy0 == ml.energy(data, lam, kind, trunc, np.zeros(shape, np.int64))
    assert e < res.energy0
    check_local_optimum(data, lam, kind, trunc, f)
    # the reference from the same start ends in a local minimum too (ties may
    # send the two runs along different moves); both are reported here
    rf, trace, _, _ = ml.alpha_expansion(data, lam, kind, trunc, np.zeros(shape, np.int64))
    print("alpha-expansion %s L=%d kind=%d warm=%d: GPU E=%.1f (%d moves, %d accepted, %d DR iterations), "
          "reference E=%.1f" % (shape, L, kind, warm, e, res.moves, res.accepted, res.dr_iters, trace[-1]))


def test_two_labels_reach_the_global_minimum(dev):
    from paper_1503_01563_amd import mc
    data, lam = problem((40, 52), 6500, 2)
    labels = Ti(np.zeros((40, 52)), dev)
    res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 0, 0.0)
    assert res.converged
    # from all-0 the move of label 1 ranges over every labelling: its exact cut
    # is the global minimum
    w, a = ml.expansion_problem(data, lam, 0, 0.0, np.zeros((40, 52), np.int64), 1)
    e_star = ml.energy(data, lam, 0, 0.0, np.zeros((40, 52), np.int64)) + oracle.mincut(w, a)[0]
    assert res.energy == e_star


def test_no_coupling_gives_pointwise_argmin(dev):
    from paper_1503_01563_amd import mc
    data, lam = problem((30, 45), 6600, 7)
    zero = [np.zeros_like(lam[0]), np.zeros_like(lam[1])]
    labels = Ti(np.zeros((30, 45)), dev)
    res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in zero], labels, 1, 2.0)
    assert res.converged and res.cycles == 2
    assert np.array_equal(labels.cpu().numpy(), np.argmin(data, axis=0))


@pytest.mark.parametrize("warm", [False, True])
def test_stereo_workload(dev, warm):
    """The 384 x 288, 16-label stereo stand-in: exact energy, local minimum."""
    from paper_1503_01563_amd import mc
    data, lam = problem((288, 384), 6000, 16)
    labels = Ti(np.zeros((288, 384)), dev)
    res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 1, 2.0, warm=warm)
    assert res.converged and res.uncertified == 0
    f = labels.cpu().numpy()
    assert res.energy == ml.energy(data, lam, 1, 2.0, f)
    check_local_optimum(data, lam, 1, 2.0, f)
    print("stereo 288x384 L=16 warm=%d: E %.1f -> %.1f, %d cycles, %d moves (%d accepted), %d DR iterations, "
          "%.1f ms" % (warm, res.energy0, res.energy, res.cycles, res.moves, res.accepted, res.dr_iters, res.ms))


def test_invalid_arguments_are_rejected(dev):
    from paper_1503_01563_amd import mc
    data, lam = problem((12, 14), 6700, 4)
    bad = np.zeros((12, 14), np.int32)
    bad[5, 7] = 4  # outside [0, n_labels)
    with pytest.raises(mc.McError):
        mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], Ti(bad, dev), 1, 2.0)
    bad[5, 7] = -1
    with pytest.raises(mc.McError):
        mc.ml_energy(T(data, dev), [T(x, dev) for x in lam], Ti(bad, dev), 1, 2.0)
    ok = Ti(np.zeros((12, 14)), dev)
    with pytest.raises(mc.McError):
        mc.expansion_problem(T(data, dev), [T(x, dev) for x in lam], ok, 4, 1, 2.0)  # alpha out of range
    with pytest.raises(mc.McError):
        mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], ok, 1, -1.0)  # negative truncation
    with pytest.raises(mc.McError):  # the warm state is a point of the two-set splitting
        mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], ok, 1, 2.0, warm=True,
                           variant=mc.VARIANT_PRODUCT)
    neg = [lam[0].copy(), lam[1]]
    neg[0][2, 3] = -1.0
    with pytest.raises(mc.McError):
        mc.alpha_expansion(T(data, dev), [T(x, dev) for x in neg], ok, 1, 2.0, validate=True)


def test_moves_under_other_outer_loops(dev):
    """The default start (warm moves) applies to the two-set splitting only;
    with another outer loop every move starts cold and the result is the same
    kind of local minimum."""
    from paper_1503_01563_amd import mc
    data, lam = problem((40, 56), 7100, 5)
    for var in (mc.VARIANT_BCD_DR, mc.VARIANT_PRODUCT):
        labels = Ti(np.zeros((40, 56)), dev)
        res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 1, 2.0, variant=var)
        assert res.converged and res.uncertified == 0, var
        f = labels.cpu().numpy()
        assert res.energy == ml.energy(data, lam, 1, 2.0, f)
        check_local_optimum(data, lam, 1, 2.0, f)


def test_degenerate_label_sets_and_shapes(dev):
    """One label: nothing can move; a single row and a single column: the
    moves are chain problems; both exact and locally minimal."""
    import torch
    from paper_1503_01563_amd import mc
    data, lam = problem((20, 24), 7000, 1)
    labels = Ti(np.zeros((20, 24)), dev)
    res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 0, 0.0)
    assert res.converged and res.accepted == 0 and res.cycles == 1 and res.energy == res.energy0
    for shape in ((1, 90), (90, 1)):
        data, lam = problem(shape, 7001, 6)
        labels = Ti(np.zeros(shape), dev)
        res = mc.alpha_expansion(T(data, dev), [T(x, dev) for x in lam], labels, 1, 2.0)
        assert res.converged
        f = labels.cpu().numpy()
        assert res.energy == ml.energy(data, lam, 1, 2.0, f)
        check_local_optimum(data, lam, 1, 2.0, f)
