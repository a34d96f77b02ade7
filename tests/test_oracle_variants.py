"""Pins of the other outer iterations (cyclic projections / BCD, alternating
projections, FISTA): certified cuts against max-flow, monotone dual
objective, AP = projected gradient, separable case, Moreau identity."""
import numpy as np
import pytest

import oracle
from oracle import variants as V
from paper_1503_01563_amd import gen

SOLVERS = {"bcd": V.bcd_solve, "ap": V.ap_solve, "fista": V.fista_solve}


@pytest.mark.parametrize("name", sorted(SOLVERS))
@pytest.mark.parametrize("shape,seed", [((24, 20), 21), ((6, 7, 5), 22)])
def test_certifies_the_minimum_cut(name, shape, seed):
    w, a = gen.iid_grid(shape, seed)
    r = SOLVERS[name](w, a, max_iters=4000, gap_tol=1e-3)
    assert r["converged"], (name, r["cert"])
    e_star = oracle.mincut(w, a, "dinic")[0]
    assert r["energy"] == e_star
    assert oracle.cut_energy(w, a, r["labels"]) == e_star


def test_bcd_dual_objective_never_increases():
    w, a = gen.iid_grid((16, 18), 23)
    r = V.bcd_solve(w, a, max_iters=40, gap_tol=0.0, history=True)
    obj = np.array(r["objective"])
    assert np.all(np.diff(obj) <= 1e-9 * np.abs(obj[:-1]) + 1e-12)


def test_fista_without_momentum_is_alternating_projections():
    # projected gradient with step 1/r is AP shifted by one iteration: AP's
    # first step projects l = 0 (y = 0), the gradient step starts from u / r
    w, a = gen.iid_grid((12, 14), 24)
    ap = V.ap_solve(w, a, max_iters=8, gap_tol=0.0)
    pg = V.fista_solve(w, a, max_iters=7, gap_tol=0.0, momentum=False)
    np.testing.assert_allclose(ap["y"], pg["y"], atol=1e-10)


def test_bcd_separable_case_is_exact_after_one_iteration():
    w, a = gen.iid_grid((15, 11), 25)
    a[1][:] = 0  # no column edges: the row prox alone solves (TV)
    r = V.bcd_solve(w, a, max_iters=1, gap_tol=1e-3)
    assert r["converged"]
    assert r["energy"] == oracle.mincut(w, a, "dinic")[0]


@pytest.mark.parametrize("axis", [0, 1])
def test_dual_sum_is_the_moreau_complement(axis):
    rng = np.random.default_rng(26)
    v = rng.normal(0, 5, size=(9, 13))
    a = [rng.uniform(0, 2, size=(9, 13)), rng.uniform(0, 2, size=(9, 13))]
    a[0][:, -1] = 0
    a[1][-1, :] = 0
    q, p = oracle.prox_family(v.shape, axis, v, a[axis])
    ps = [np.zeros_like(v), np.zeros_like(v)]
    ps[axis] = p
    np.testing.assert_allclose(V.dual_sum(a, ps), v - q, atol=1e-9)
