"""Pins of the 8-connected reference: chain families against the edge set,
energies against the 4-connected C oracle and hand counts, max-flow against
brute force, and the splitting's certified cuts against max-flow."""
import numpy as np
import pytest

import oracle
from oracle import grid8


def grid8_problem(shape, seed, w_max=20, a_max=10):
    rng = np.random.default_rng(seed)
    H, W = shape
    w = rng.integers(-w_max, w_max + 1, size=shape).astype(np.float64)
    a = [rng.integers(0, a_max + 1, size=shape).astype(np.float64) for _ in range(4)]
    a[0][:, -1] = 0
    a[1][-1, :] = 0
    for k in (2, 3):
        a[k][-1, :] = 0
        a[k][:, -1] = 0
    return w, a


@pytest.mark.parametrize("shape", [(2, 2), (3, 5), (6, 4), (7, 9)])
def test_families_partition_the_edges(shape):
    H, W = shape
    w, a = grid8_problem(shape, 1)
    fams = grid8.families(H, W, a)
    # every edge of the grid is an edge of exactly one chain, with its weight
    seen = {}
    for j, fam in enumerate(fams):
        used = set()
        for verts, wts in fam:
            assert len(wts) == len(verts) - 1
            assert not used & set(verts.tolist()), "chains of one family share a vertex"
            used |= set(verts.tolist())
            for k in range(len(wts)):
                key = tuple(sorted((int(verts[k]), int(verts[k + 1]))))
                assert key not in seen
                seen[key] = wts[k]
    expect = {}
    for u, v, wt in grid8.edge_list(H, W, a):
        for x, y, z in zip(u, v, wt):
            expect[tuple(sorted((int(x), int(y))))] = z
    assert seen.keys() == expect.keys()
    assert all(seen[k] == expect[k] for k in seen)


def test_energy_hand_count():
    # 2 x 2, labels {(0,0), (1,1)}: the four axis edges are cut; the diagonal
    # (0,0)-(1,1) has both ends in S, the anti-diagonal (1,0)-(0,1) neither
    w = np.array([[1.0, -2.0], [3.0, -4.0]])
    a = [np.array([[5.0, 0], [7.0, 0]]), np.array([[11.0, 13.0], [0, 0]]),
         np.array([[17.0, 0], [0, 0]]), np.array([[19.0, 0], [0, 0]])]
    lab = np.array([[1, 0], [0, 1]])
    assert grid8.cut_energy(w, a, lab) == 1 - 4 + 5 + 7 + 11 + 13
    # {(0,0), (0,1)}: the vertical edges and both diagonals are cut
    lab2 = np.array([[1, 1], [0, 0]])
    assert grid8.cut_energy(w, a, lab2) == 1 - 2 + 11 + 13 + 17 + 19


def test_energy_matches_four_connected_oracle():
    w, a = grid8_problem((9, 7), 2)
    a[2][:] = 0
    a[3][:] = 0
    lab = np.random.default_rng(3).integers(0, 2, size=(9, 7)).astype(np.uint8)
    assert grid8.cut_energy(w, a, lab) == oracle.cut_energy(w, a[:2], lab)


@pytest.mark.parametrize("shape,seed", [((3, 4), 4), ((4, 4), 5), ((2, 7), 6), ((4, 3), 7)])
def test_mincut_matches_bruteforce(shape, seed):
    w, a = grid8_problem(shape, seed, w_max=9, a_max=6)
    e_star, S = grid8.mincut(w, a)
    e_bf, _ = grid8.bruteforce(w, a)
    assert e_star == e_bf
    assert grid8.cut_energy(w, a, S) == e_star


def test_mincut_matches_four_connected_dinic():
    w, a = grid8_problem((20, 17), 8)
    a[2][:] = 0
    a[3][:] = 0
    assert grid8.mincut(w, a)[0] == oracle.mincut(w, a[:2], "dinic")[0]


@pytest.mark.parametrize("shape,seed", [((8, 9), 9), ((12, 10), 10), ((1, 6), 11), ((6, 1), 12)])
def test_splitting_certifies_the_minimum_cut(shape, seed):
    w, a = grid8_problem(shape, seed)
    r = grid8.dr_solve(w, a, max_iters=600, gap_tol=1e-3)
    assert r["converged"]
    e_star, _ = grid8.mincut(w, a)
    assert r["energy"] == e_star
    assert grid8.cut_energy(w, a, r["labels"]) == e_star
