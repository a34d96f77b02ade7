"""Multi-label energies by alpha-expansion: plain FP64 reference (test
infrastructure only; nothing in the GPU library calls this module).

Sec. 4.4 of the paper reduces multi-label energy minimisation to a series of
binary cut problems by move-making (alpha-expansion of Boykov, Veksler and
Zabih, 2001), and Sec. 6.1 solves a 4-connected stereo task that way with the
r = 2 dual.  On an H x W grid with labels f_i in {0..L-1}:

    E(f) = sum_i D[f_i, i] + sum_{edges e = (u, v)} lam_e V(f_u, f_v)

lam[0][r][c] weighs (r, c) - (r, c+1) (last column 0), lam[1][r][c] weighs
(r, c) - (r+1, c) (last row 0); V is a metric: Potts V(a, b) = [a != b] or the
truncated linear V(a, b) = min(|a - b|, T).

Expansion move for label alpha: every pixel either keeps f_i (x_i = 0) or
takes alpha (x_i = 1).  With A = V(f_u, f_v), B = V(f_u, alpha),
C = V(alpha, f_v) and V(alpha, alpha) = 0, the edge term of the move is
lam (A + (C - A) x_u - C x_v + k (1 - x_u) x_v) with k = B + C - A >= 0 (triangle
inequality), and k (1 - x_u) x_v = k/2 |x_u - x_v| + k/2 (x_v - x_u).  So the
move is the cut problem of this package, E(f') = E(f) + E_bin(S) with S the
switching pixels and
    w_i  = D[alpha, i] - D[f_i, i] + sum over edges of the terms below,
    u:  lam (C - A - B) / 2,   v:  lam (B - A - C) / 2,   a_e = lam (B + C - A) / 2.
The move taken is the minimal optimal set of that problem (max-flow), accepted
when it lowers the energy; a cycle visits alpha = 0..L-1 in order, and the loop
stops after a cycle without an accepted move.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import cut_energy, mincut

POTTS = 0
TRUNC_LINEAR = 1


def vdist(kind, trunc, a, b):
    """V(a, b) elementwise (FP64)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if kind == POTTS:
        return (a != b).astype(np.float64)
    return np.minimum(np.abs(a - b).astype(np.float64), float(trunc))


def energy(data, lam, kind, trunc, f):
    """E(f) in FP64 by its definition."""
    data = np.asarray(data, np.float64)
    f = np.asarray(f, np.int64)
    H, W = f.shape
    e = float(np.take_along_axis(data, f[None], axis=0).sum())
    lx = np.asarray(lam[0], np.float64)
    ly = np.asarray(lam[1], np.float64)
    e += float(np.sum(lx[:, :-1] * vdist(kind, trunc, f[:, :-1], f[:, 1:])))
    e += float(np.sum(ly[:-1, :] * vdist(kind, trunc, f[:-1, :], f[1:, :])))
    return e


def expansion_problem(data, lam, kind, trunc, f, alpha):
    """Binary problem (w, [a_x, a_y]) of the alpha-expansion move from f."""
    data = np.asarray(data, np.float64)
    f = np.asarray(f, np.int64)
    H, W = f.shape
    w = data[alpha] - np.take_along_axis(data, f[None], axis=0)[0]
    a = [np.zeros((H, W)), np.zeros((H, W))]
    for j, (su, sv) in enumerate((((slice(None), slice(None, -1)), (slice(None), slice(1, None))),
                                  ((slice(None, -1), slice(None)), (slice(1, None), slice(None))))):
        lj = np.asarray(lam[j], np.float64)[su]
        fu, fv = f[su], f[sv]
        A = vdist(kind, trunc, fu, fv)
        B = vdist(kind, trunc, fu, alpha)
        C = vdist(kind, trunc, alpha, fv)
        a[j][su] = lj * (B + C - A) / 2
        w[su] += lj * (C - A - B) / 2
        w[sv] += lj * (B - A - C) / 2
    return w, a


def apply_move(f, S, alpha):
    f = np.array(f, np.int64, copy=True)
    f[np.asarray(S, bool)] = alpha
    return f


def alpha_expansion(data, lam, kind, trunc, f0, max_cycles=50, skip_unchanged=False):
    """Alpha-expansion from f0 with exact moves (minimal optimal sets by
    max-flow).  Returns (f, energies after each accepted move, cycles, moves).

    skip_unchanged: do not solve the move of a label when no move has been
    applied since that label's previous move.  The labels are then the same
    as at that move, which was either rejected (an exact move finds no
    improvement again) or applied (the expansions of alpha from its result
    are expansions from the labels before it, so none improves on it), so the
    applied moves and the result are those of the plain loop."""
    data = np.asarray(data, np.float64)
    L = data.shape[0]
    f = np.array(f0, np.int64, copy=True)
    e = energy(data, lam, kind, trunc, f)
    trace = [e]
    moves = 0
    cycles = 0
    applied = 0
    seen = [-1] * L  # applied-move count when each label's move was last solved
    for _ in range(max_cycles):
        cycles += 1
        improved = False
        for alpha in range(L):
            if skip_unchanged and seen[alpha] == applied:
                continue
            w, a = expansion_problem(data, lam, kind, trunc, f, alpha)
            eb, S, _ = mincut(w, a)
            moves += 1
            if eb < 0:
                f = apply_move(f, S, alpha)
                e += eb
                trace.append(e)
                improved = True
                applied += 1
            seen[alpha] = applied
        if not improved:
            break
    return f, trace, cycles, moves


def bruteforce(data, lam, kind, trunc):
    """Minimum of E over all L^n labellings (tiny grids): (E*, one minimiser)."""
    data = np.asarray(data, np.float64)
    L, H, W = data.shape
    best, arg = np.inf, None
    for labs in itertools.product(range(L), repeat=H * W):
        f = np.array(labs, np.int64).reshape(H, W)
        e = energy(data, lam, kind, trunc, f)
        if e < best:
            best, arg = e, f
    return best, arg


def best_move_bruteforce(data, lam, kind, trunc, f, alpha):
    """Smallest E(f') - E(f) over all 2^n moves of label alpha (tiny grids)."""
    f = np.asarray(f, np.int64)
    e0 = energy(data, lam, kind, trunc, f)
    best = np.inf
    for bits in itertools.product((0, 1), repeat=f.size):
        S = np.array(bits, bool).reshape(f.shape)
        best = min(best, energy(data, lam, kind, trunc, apply_move(f, S, alpha)) - e0)
    return best


def move_energy(w, a, S):
    """E_bin(S) of a move problem (the cut energy of the package's form)."""
    return cut_energy(w, a, S)
