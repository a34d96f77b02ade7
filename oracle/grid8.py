"""8-connected 2D grids: plain FP64 reference (test infrastructure only).

Nothing in the GPU library calls this module.

Edges of an H x W grid, weights stored per vertex / cell (r, c):
  a[0][r][c]  (r, c) - (r, c+1)        along W      (last column 0)
  a[1][r][c]  (r, c) - (r+1, c)        along H      (last row 0)
  a[2][r][c]  (r, c) - (r+1, c+1)      diagonal     (last row and column 0)
  a[3][r][c]  (r+1, c) - (r, c+1)      anti-diagonal (last row and column 0)
E(S) = sum_{i in S} w_i + sum_edges a_e [exactly one end in S]   (problem (D)).

Chain families (Sec. 3.1 and Fig. 1 of the paper: rows, columns and
zig-zag paths).  The strip of rows r and r+1 holds two zig-zag paths over
the columns q = 0..W-1: path 0 visits row r + (q mod 2), path 1 visits row
r + 1 - (q mod 2).  Edge q of path 0 is the diagonal of cell (r, q) when q is
even and its anti-diagonal when q is odd; path 1 the other way round.  The
two paths share no vertex and together hold every diagonal edge of the
strip once.  Strips with even r form one family, odd r another: four
families in all, each a union of vertex-disjoint chains (vertices on no chain
of a family are left alone by its prox).

The splitting is Douglas-Rachford in the product space (Sec. 4.3) with
r = 4, exactly as for the 3D grids; the certificate and the threshold ladder
are those of the 4-connected case.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import tv1d

N_TAU = 9


def tau_ladder(tau0):
    return [tau0 * f for f in (1.0, 1e-1, 1e-2, 1e-3, 0.0, -1e-3, -1e-2, -1e-1, -1.0)]


def edge_list(H, W, a):
    """(u, v, weight) index arrays of every edge with its weight."""
    idx = np.arange(H * W).reshape(H, W)
    out = []
    us, vs = idx[:, :-1], idx[:, 1:]
    out.append((us.ravel(), vs.ravel(), np.asarray(a[0], np.float64)[:, :-1].ravel()))
    us, vs = idx[:-1, :], idx[1:, :]
    out.append((us.ravel(), vs.ravel(), np.asarray(a[1], np.float64)[:-1, :].ravel()))
    us, vs = idx[:-1, :-1], idx[1:, 1:]
    out.append((us.ravel(), vs.ravel(), np.asarray(a[2], np.float64)[:-1, :-1].ravel()))
    us, vs = idx[1:, :-1], idx[:-1, 1:]
    out.append((us.ravel(), vs.ravel(), np.asarray(a[3], np.float64)[:-1, :-1].ravel()))
    return out


def cut_energy(w, a, labels):
    H, W = np.shape(w)
    S = np.asarray(labels, bool).ravel()
    e = float(np.sum(np.asarray(w, np.float64).ravel()[S]))
    for u, v, wt in edge_list(H, W, a):
        e += float(np.sum(wt[S[u] != S[v]]))
    return e


def bruteforce(w, a):
    """Minimum over all 2^n labellings (n <= 20): (E*, one minimiser)."""
    H, W = np.shape(w)
    n = H * W
    assert n <= 20
    best, arg = np.inf, None
    for bits in itertools.product((0, 1), repeat=n):
        lab = np.array(bits, np.uint8).reshape(H, W)
        e = cut_energy(w, a, lab)
        if e < best:
            best, arg = e, lab
    return best, arg


def mincut(w, a, scale=256):
    """Exact minimum cut by max-flow on the s-t graph of (D) (scipy's
    maximum_flow on capacities scaled by `scale` to integers; the data must
    be multiples of 1/scale).  Returns (E*, minimal optimal set)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow
    H, W = np.shape(w)
    n = H * W
    wf = np.asarray(w, np.float64).ravel() * scale
    s, t = n, n + 1
    rows, cols, caps = [], [], []
    for u, v, wt in edge_list(H, W, a):
        m = wt > 0
        c = wt[m] * scale
        rows += [u[m], v[m]]
        cols += [v[m], u[m]]
        caps += [c, c]
    pos, neg = wf > 0, wf < 0
    rows += [np.nonzero(pos)[0], np.full(int(neg.sum()), s)]
    cols += [np.full(int(pos.sum()), t), np.nonzero(neg)[0]]
    caps += [wf[pos], -wf[neg]]
    r, c, cap = np.concatenate(rows), np.concatenate(cols), np.concatenate(caps)
    capi = np.rint(cap)
    if not np.all(capi == cap) or cap.max(initial=0) >= 2 ** 31:
        raise ValueError("capacities must be integers after scaling")
    G = csr_matrix((capi.astype(np.int32), (r, c)), shape=(n + 2, n + 2))
    G.sum_duplicates()
    res = maximum_flow(G, s, t)
    e_star = res.flow_value / scale + float(np.sum(np.minimum(np.asarray(w, np.float64), 0)))
    # minimal optimal set: reachable from s in the residual graph
    F = res.flow.tocsr()
    resid = (G - F).tocsr()
    resid.data[resid.data < 0] = 0
    resid.eliminate_zeros()
    reach = np.zeros(n + 2, bool)
    reach[s] = True
    stack = [s]
    while stack:
        u = stack.pop()
        for v in resid.indices[resid.indptr[u]:resid.indptr[u + 1]]:
            if not reach[v]:
                reach[v] = True
                stack.append(v)
    return e_star, reach[:n].reshape(H, W).astype(np.uint8)


def families(H, W, a):
    """The four chain families: lists of (vertex indices, edge weights)."""
    a = [np.asarray(x, np.float64) for x in a]
    fams = [[], [], [], []]
    for r in range(H):
        fams[0].append((r * W + np.arange(W), a[0][r, :W - 1]))
    for c in range(W):
        fams[1].append((np.arange(H) * W + c, a[1][:H - 1, c]))
    q = np.arange(W)
    for r in range(H - 1):
        for path in (0, 1):
            rows = r + ((q + path) & 1)
            verts = rows * W + q
            diag = ((q[:-1] + path) & 1) == 0
            wts = np.where(diag, a[2][r, :W - 1], a[3][r, :W - 1])
            fams[2 + (r & 1)].append((verts, wts))
    return fams


def prox_family(fam, v):
    """Prox of one family's TV at v (identity off its chains), and each chain's duals."""
    x = np.array(v, np.float64, copy=True)
    duals = []
    for verts, wts in fam:
        xc, p = tv1d(v[verts], wts)
        x[verts] = xc
        duals.append(p)
    return x, duals


def dual_vector(fam, duals, n):
    """sum over the family's chains of D^T p, (D^T p)_k = p_{k-1} - p_k along a chain."""
    y = np.zeros(n)
    for (verts, _), p in zip(fam, duals):
        m = len(verts)
        contrib = np.zeros(m)
        contrib[1:] += p
        contrib[:-1] -= p
        y[verts] += contrib
    return y


def certificate(w, a, fams, duals, tau0):
    """Clipped duals -> y in K, LB, primal -w - y, ladder energies; returns
    (cert, energy, lb, labels)."""
    H, W = np.shape(w)
    n = H * W
    wf = np.asarray(w, np.float64).ravel()
    y = np.zeros(n)
    for fam, ds in zip(fams, duals):
        clipped = [np.clip(p, -wts, wts) for (_, wts), p in zip(fam, ds)]
        y += dual_vector(fam, clipped, n)
    lb = float(np.sum(np.minimum(y + wf, 0.0)))
    x = -wf - y
    best, lab = np.inf, None
    for tau in tau_ladder(tau0):
        S = (x > tau).reshape(H, W)
        e = cut_energy(w, a, S)
        if e < best:
            best, lab = e, S.astype(np.uint8)
    return best - lb, best, lb, lab, x.reshape(H, W)


def dr_solve(w, a, max_iters=500, gap_tol=1e-3, tau0=1e-3, z0=None, check_every=1):
    """Product-space Douglas-Rachford over the four families (Sec. 4.3):
    q_j = prox_j(z_j), y_j = z_j - q_j, z_j <- y_j - (2Y - Z + w)/4 with
    Y = sum y_j, Z = sum z_j; starts from z = 0.  Returns a dict."""
    H, W = np.shape(w)
    n = H * W
    R = 4
    wf = np.asarray(w, np.float64).ravel()
    fams = families(H, W, a)
    z = np.zeros((R, n)) if z0 is None else np.array(z0, np.float64).reshape(R, n)
    out = None
    for it in range(1, max_iters + 1):
        ys, duals = [], []
        for j in range(R):
            q, d = prox_family(fams[j], z[j])
            ys.append(z[j] - q)
            duals.append(d)
        Y, Z = np.sum(ys, axis=0), np.sum(z, axis=0)
        z = np.array([ys[j] - (2 * Y - Z + wf) / R for j in range(R)])
        if it % check_every and it != max_iters:
            continue
        cert, e, lb, lab, x = certificate(w, a, fams, duals, tau0)
        out = {"iters": it, "cert": cert, "energy": e, "lower_bound": lb, "labels": lab, "x": x, "z": z}
        if cert < gap_tol:
            out["converged"] = True
            return out
    out["converged"] = False
    return out
