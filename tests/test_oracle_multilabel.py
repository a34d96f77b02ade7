"""Pins of the alpha-expansion reference (oracle/multilabel.py) against the
definition of the multi-label energy and brute force (Sec. 4.4 and 6.1 of the
paper: multi-label problems solved as a series of binary cuts)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import multilabel as ml
from paper_1503_01563_amd import gen


def tiny(seed, H=2, W=3, L=3, kind=ml.TRUNC_LINEAR, lam_max=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    data = rng.integers(0, 6, size=(L, H, W)).astype(np.float64)
    lx = rng.integers(0, lam_max + 1, size=(H, W)).astype(np.float64)
    ly = rng.integers(0, lam_max + 1, size=(H, W)).astype(np.float64)
    lx[:, -1] = 0
    ly[-1, :] = 0
    f = rng.integers(0, L, size=(H, W))
    return data, [lx, ly], f


def test_energy_hand_count():
    # 1 x 3 chain, labels (0, 2, 2), truncated linear T = 1, lam = (2, 5)
    data = np.zeros((3, 1, 3))
    data[0, 0, 0] = 1.0
    data[2, 0, 1] = 4.0
    data[2, 0, 2] = 7.0
    lx = np.array([[2.0, 5.0, 0.0]])
    ly = np.zeros((1, 3))
    f = np.array([[0, 2, 2]])
    # data 1 + 4 + 7, edges 2 min(2, 1) + 5 min(0, 1)
    assert ml.energy(data, [lx, ly], ml.TRUNC_LINEAR, 1, f) == 12.0 + 2.0
    # Potts: the same edges cost 2 [0 != 2] + 5 [2 != 2]
    assert ml.energy(data, [lx, ly], ml.POTTS, 0, f) == 12.0 + 2.0


@pytest.mark.parametrize("kind", [ml.POTTS, ml.TRUNC_LINEAR])
@pytest.mark.parametrize("seed", range(6))
def test_move_reduction_is_exact(kind, seed):
    """E(f with S switched to alpha) = E(f) + E_bin(S) for every S and alpha:
    the binary problem is the move, term by term."""
    data, lam, f = tiny(seed, kind=kind)
    e0 = ml.energy(data, lam, kind, 2, f)
    for alpha in range(data.shape[0]):
        w, a = ml.expansion_problem(data, lam, kind, 2, f, alpha)
        assert np.all(a[0] >= 0) and np.all(a[1] >= 0)  # metric V: the move is a cut
        assert np.all(a[0][:, -1] == 0) and np.all(a[1][-1, :] == 0)
        for bits in itertools.product((0, 1), repeat=f.size):
            S = np.array(bits, np.uint8).reshape(f.shape)
            lhs = ml.energy(data, lam, kind, 2, ml.apply_move(f, S, alpha))
            assert lhs == e0 + ml.move_energy(w, a, S)


def test_two_labels_one_move_is_the_optimum():
    """With two labels an expansion from all-0 ranges over every labelling, so
    the first move of label 1 already reaches the global minimum."""
    for seed in range(5):
        data, lam, _ = tiny(100 + seed, H=3, W=3, L=2, kind=ml.POTTS)
        e_star, _ = ml.bruteforce(data, lam, ml.POTTS, 0)
        w, a = ml.expansion_problem(data, lam, ml.POTTS, 0, np.zeros((3, 3), np.int64), 1)
        eb, S, _ = oracle.mincut(w, a)
        assert ml.energy(data, lam, ml.POTTS, 0, np.zeros((3, 3))) + eb == e_star
        f, trace, _, _ = ml.alpha_expansion(data, lam, ml.POTTS, 0, np.zeros((3, 3), np.int64))
        assert trace[-1] == e_star == ml.energy(data, lam, ml.POTTS, 0, f)


def test_no_coupling_gives_pointwise_argmin():
    rng = np.random.Generator(np.random.PCG64(7))
    data = rng.integers(0, 9, size=(5, 6, 7)).astype(np.float64)
    lam = [np.zeros((6, 7)), np.zeros((6, 7))]
    f, _, cycles, _ = ml.alpha_expansion(data, lam, ml.TRUNC_LINEAR, 2, np.zeros((6, 7), np.int64))
    assert np.array_equal(f, np.argmin(data, axis=0))  # first minimiser: ties never switch
    assert cycles == 2  # one improving cycle, one that confirms


@pytest.mark.parametrize("kind", [ml.POTTS, ml.TRUNC_LINEAR])
@pytest.mark.parametrize("seed", range(4))
def test_local_optimum_and_bounds(kind, seed):
    """The result admits no improving expansion (brute force over all 2^n
    moves of every label), the energy never rises, and for Potts it is within
    the factor 2 of the global minimum that expansion guarantees."""
    data, lam, f0 = tiny(200 + seed, H=2, W=4, L=3, kind=kind)
    f, trace, _, _ = ml.alpha_expansion(data, lam, kind, 2, f0)
    assert all(b < a for a, b in zip(trace, trace[1:]))
    assert trace[-1] == ml.energy(data, lam, kind, 2, f)
    for alpha in range(3):
        assert ml.best_move_bruteforce(data, lam, kind, 2, f, alpha) >= 0
    e_star, _ = ml.bruteforce(data, lam, kind, 2)
    assert e_star <= trace[-1]
    if kind == ml.POTTS:
        assert trace[-1] <= 2 * e_star


def test_generator_shapes_and_exactness():
    data, lam, true = gen.stereo_labels((24, 32), 6000, n_labels=8)
    assert data.shape == (8, 24, 32) and data.dtype == np.float32
    assert np.all(data == np.rint(data)) and data.min() >= 0
    assert np.all(lam[0][:, -1] == 0) and np.all(lam[1][-1, :] == 0)
    assert true.min() >= 0 and true.max() < 8
    f, trace, _, _ = ml.alpha_expansion(data, lam, ml.TRUNC_LINEAR, 2, np.zeros((24, 32), np.int64))
    assert trace[-1] < trace[0]
    assert trace[-1] == ml.energy(data, lam, ml.TRUNC_LINEAR, 2, f)


@pytest.mark.parametrize("kind", [ml.POTTS, ml.TRUNC_LINEAR])
@pytest.mark.parametrize("seed", range(3))
def test_skipping_unchanged_moves_changes_nothing(kind, seed):
    """Skipping the move of a label while no move has been applied since its
    previous one gives the same applied moves, energies and labels as the
    plain loop, with fewer moves solved."""
    data, lam, _ = gen.stereo_labels((14, 18), 6800 + seed, n_labels=6)
    data = data.astype(np.float64)
    lam = [x.astype(np.float64) for x in lam]
    f0 = np.zeros((14, 18), np.int64)
    f1, t1, c1, m1 = ml.alpha_expansion(data, lam, kind, 2, f0)
    f2, t2, c2, m2 = ml.alpha_expansion(data, lam, kind, 2, f0, skip_unchanged=True)
    assert np.array_equal(f1, f2) and t1 == t2 and c1 == c2
    assert m2 < m1
    # the final cycle of the plain loop rejects every label; with the skip only
    # the labels solved before the last applied move are solved again
    assert m1 == c1 * 6
