"""Other outer iterations on the same chain proxes (test infrastructure only).

Sec. 4.1-4.2 of the paper, written in this package's sign (u = -w, primal
x = u - sum_j y_j, y_j in K_j, the dual problem min_{y in K} 1/2 |u - sum_j y_j|^2):

  block coordinate descent / cyclic projections (Sec. 4.1): for i = 1..r in
      turn, y_i <- Pi_{K_i}(u - sum_{j != i} y_j); with v = x + y_i this is
      x <- prox_i(v), y_i <- v - x;
  alternating projections in the product space (Sec. 4.2): y_j <- Pi_{K_j}(l_j)
      for all j, then l <- Pi_L(y), i.e. l_j = y_j + (u - sum_k y_k) / r;
  FISTA on the smooth dual (Sec. 4.1; the gradient of the objective in y_j
      is -x and its Lipschitz constant is r): y_j <- Pi_{K_j}(yt_j + xt / r)
      with xt = u - sum_j yt_j at the extrapolated point
      yt = y_k + (t_k - 1) / t_{k+1} (y_k - y_{k-1}),
      t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, t_1 = 1.
Pi_{K_j}(v) = v - prox_j(v) (Moreau).  Every projection comes from the chain
prox of `prox_family`, whose edge duals also give the certificate: y from
the last duals of every family, clipped (so y is in K exactly), LB(y), the
primal -w - y and the energies of the threshold ladder, as for the splitting.
"""
from __future__ import annotations

import numpy as np

from . import cut_energy, lower_bound, prox_family

TAU_FACTORS = (1.0, 1e-1, 1e-2, 1e-3, 0.0, -1e-3, -1e-2, -1e-1, -1.0)


def _axis_np(nd, j):
    return nd - 1 - j  # grid axis j (0 = W) -> numpy axis


def dual_sum(a, p):
    """sum_j D_j^T clip(p_j), (D^T p)_i = p_{i - e_j} - p_i along axis j."""
    nd = len(a)
    y = np.zeros(np.shape(p[0]))
    for j in range(nd):
        pj = np.clip(np.asarray(p[j], np.float64), -np.asarray(a[j], np.float64), np.asarray(a[j], np.float64))
        ax = _axis_np(nd, j)
        y -= pj
        sl_dst = [slice(None)] * nd
        sl_src = [slice(None)] * nd
        sl_dst[ax] = slice(1, None)
        sl_src[ax] = slice(None, -1)
        y[tuple(sl_dst)] += pj[tuple(sl_src)]
    return y


def certify(w, a, p, tau0=1e-3):
    """(cert, energy, lb, labels, x) from the edge duals p of every family."""
    w = np.asarray(w, np.float64)
    lb, _ = lower_bound(w, a, [np.asarray(x, np.float64) for x in p])
    x = -w - dual_sum(a, p)
    best, lab = np.inf, None
    for f in TAU_FACTORS:
        S = (x > tau0 * f).astype(np.uint8)
        e = cut_energy(w, a, S)
        if e < best:
            best, lab = e, S
    return best - lb, best, lb, lab, x


def _prox(w, j, v, a):
    return prox_family(np.shape(w), j, v, np.asarray(a[j], np.float64))


def _result(it, cert, e, lb, lab, x, converged, extra):
    out = {"iters": it, "cert": cert, "energy": e, "lower_bound": lb, "labels": lab, "x": x,
           "converged": converged}
    out.update(extra)
    return out


def bcd_solve(w, a, max_iters=500, gap_tol=1e-3, tau0=1e-3, check_every=1, history=False):
    w = np.asarray(w, np.float64)
    nd = w.ndim
    u = -w
    y = np.zeros((nd,) + w.shape)
    x = u.copy()
    p = [np.zeros(w.shape) for _ in range(nd)]
    objective = []
    res = None
    for it in range(1, max_iters + 1):
        for i in range(nd):
            v = x + y[i]
            x, p[i] = _prox(w, i, v, a)
            y[i] = v - x
        if history:
            objective.append(0.5 * float(np.sum((u - y.sum(axis=0)) ** 2)))
        if it % check_every and it != max_iters:
            continue
        cert, e, lb, lab, xc = certify(w, a, p, tau0)
        res = (it, cert, e, lb, lab, xc)
        if cert < gap_tol:
            return _result(*res, True, {"y": y, "objective": objective})
    return _result(*res, False, {"y": y, "objective": objective})


def ap_solve(w, a, max_iters=500, gap_tol=1e-3, tau0=1e-3, check_every=1):
    w = np.asarray(w, np.float64)
    nd = w.ndim
    u = -w
    lam = np.zeros((nd,) + w.shape)
    y = np.zeros_like(lam)
    p = [None] * nd
    res = None
    for it in range(1, max_iters + 1):
        for j in range(nd):
            q, p[j] = _prox(w, j, lam[j], a)
            y[j] = lam[j] - q
        x = u - y.sum(axis=0)
        lam = y + x / nd
        if it % check_every and it != max_iters:
            continue
        cert, e, lb, lab, xc = certify(w, a, p, tau0)
        res = (it, cert, e, lb, lab, xc)
        if cert < gap_tol:
            return _result(*res, True, {"y": y, "lam": lam})
    return _result(*res, False, {"y": y, "lam": lam})


def fista_solve(w, a, max_iters=500, gap_tol=1e-3, tau0=1e-3, check_every=1, momentum=True):
    w = np.asarray(w, np.float64)
    nd = w.ndim
    u = -w
    y = np.zeros((nd,) + w.shape)
    y_prev = y.copy()
    t = 1.0
    p = [None] * nd
    res = None
    for it in range(1, max_iters + 1):
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_next if momentum else 0.0
        yt = y + beta * (y - y_prev)
        xt = u - yt.sum(axis=0)
        y_new = np.empty_like(y)
        for j in range(nd):
            v = yt[j] + xt / nd
            q, p[j] = _prox(w, j, v, a)
            y_new[j] = v - q
        y_prev, y, t = y, y_new, t_next
        if it % check_every and it != max_iters:
            continue
        cert, e, lb, lab, xc = certify(w, a, p, tau0)
        res = (it, cert, e, lb, lab, xc)
        if cert < gap_tol:
            return _result(*res, True, {"y": y})
    return _result(*res, False, {"y": y})
