"""Seeded synthetic inputs: grid cut problems (unaries w, edge weights a).

This module only draws inputs; it holds none of the solver's arithmetic, and
both the GPU path and the CPU checker are fed from it.  All draws use numpy's
PCG64 with an explicit seed.  Arrays are float32 holding values that are exact
in FP32 and FP64 (integers, or multiples of 2^-8), so energies are exact sums.

Layout: ``w`` has the grid shape ``(H, W)`` or ``(D, H, W)``, W contiguous;
``a`` is a list with one array per axis (0 = W, 1 = H, 2 = D) of the same
shape, ``a[j][i]`` the weight of edge ``(i, i + stride_j)``; the last slice
along axis ``j`` is zero.

Workloads (the paper's maxflow-benchmark volumes are not available; these
stand in for them):
  * ``iid_grid``      -- integer unaries U{-20..20}, integer weights U{0..10}.
  * ``ellipse_grid``  -- two-region piecewise-constant image (random ellipses
                         or ellipsoids, intensities 0.3 / 0.7) plus Gaussian
                         noise; w = cost of the foreground label (negative
                         log-likelihood ratio), a = lam * exp(-dI^2 / (2 0.1^2)),
                         both rounded to multiples of 2^-8.
  * ``batch_sizes``   -- uneven (H, W) pairs for batched solves.
  * ``ellipse_sequence``, ``edit_sequence`` -- frames of drifting ellipses, and
                         an integer grid whose unaries are partly redrawn per
                         frame (related problems for reusing one frame's dual
                         in the next).
  * ``stereo_labels``  -- a multi-label problem shaped like a small stereo
                         task (piecewise-constant label map: a tilted
                         background plane and objects at constant labels,
                         noisy observed labels with outliers): integer data
                         costs D[l] = min(|obs - l|, t_data), integer edge
                         weights that drop across intensity edges.
"""
from __future__ import annotations

import numpy as np

DYADIC = 2.0 ** -8


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _zero_last(a, axis_from_end):
    """Zero the last slice along the axis (0 = W = last numpy axis)."""
    idx = [slice(None)] * a.ndim
    idx[a.ndim - 1 - axis_from_end] = -1
    a[tuple(idx)] = 0
    return a


def iid_grid(shape, seed, w_max=20, a_max=10):
    """Integer unaries U{-w_max..w_max} and weights U{0..a_max} on every axis."""
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    w = rng.integers(-w_max, w_max + 1, size=shape).astype(np.float32)
    a = []
    for j in range(len(shape)):
        aj = rng.integers(0, a_max + 1, size=shape).astype(np.float32)
        a.append(_zero_last(aj, j))
    return w, a


def _quantise(x):
    return (np.round(np.asarray(x, np.float64) / DYADIC) * DYADIC).astype(np.float32)


def _ellipses(rng, shape, k_range=(3, 8), axes_frac=(0.05, 0.25)):
    """Random ellipses (ellipsoids): list of (centre, semi-axes, rotation)."""
    nd = len(shape)
    k = int(rng.integers(k_range[0], k_range[1] + 1))
    ext = np.array(shape, dtype=np.float64)
    out = []
    for _ in range(k):
        centre = rng.uniform(0, 1, size=nd) * ext
        if nd == 2:
            semi = rng.uniform(axes_frac[0], axes_frac[1], size=2) * min(shape)
            ang = rng.uniform(0, np.pi)
            c, s = np.cos(ang), np.sin(ang)
            rot = np.array([[c, -s], [s, c]])
        else:
            semi = rng.uniform(axes_frac[0], axes_frac[1], size=3) * ext
            q, r = np.linalg.qr(rng.normal(size=(3, 3)))
            rot = q * np.sign(np.diag(r))
        out.append((centre, semi, rot))
    return out


def _render(shape, ellipses, rng, sigma):
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) + 0.5 for s in shape], indexing="ij")
    coords = np.stack([g.ravel() for g in grids], axis=1)  # (n, nd), numpy axis order
    inside = np.zeros(coords.shape[0], dtype=bool)
    for centre, semi, rot in ellipses:
        d = (coords - centre) @ rot
        inside |= np.sum((d / semi) ** 2, axis=1) <= 1.0
    img = np.where(inside, 0.7, 0.3).reshape(shape)
    return img + rng.normal(0.0, sigma, size=shape)


def ellipse_image(shape, seed, sigma=0.15, k_range=(3, 8), axes_frac=(0.05, 0.25)):
    """Noisy two-region image in [D][H][W] or [H][W]: 0.7 inside random ellipses."""
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    return _render(shape, _ellipses(rng, shape, k_range, axes_frac), rng, sigma)


def _image_to_grid(img, lam, sigma, beta_sigma):
    w = ((img - 0.7) ** 2 - (img - 0.3) ** 2) / (2.0 * sigma ** 2)
    a = []
    nd = img.ndim
    for j in range(nd):
        ax = nd - 1 - j  # numpy axis of grid axis j
        nxt = np.roll(img, -1, axis=ax)
        aj = lam * np.exp(-((nxt - img) ** 2) / (2.0 * beta_sigma ** 2))
        a.append(_zero_last(_quantise(aj), j))
    return _quantise(w), a


def ellipse_grid(shape, seed, lam=2.0, sigma=0.15, beta_sigma=0.1):
    """Segmentation-shaped cut problem from a noisy ellipse (ellipsoid) image."""
    return _image_to_grid(ellipse_image(shape, seed, sigma=sigma), lam, sigma, beta_sigma)


def ellipse_grid8(shape, seed, lam=2.0, sigma=0.15, beta_sigma=0.1):
    """8-connected version of `ellipse_grid` (2D): the same image, unaries and
    axis weights, plus diagonal weights lam / sqrt(2) * exp(-dI^2 / (2 0.1^2))
    across each cell's diagonal (r,c)-(r+1,c+1) and anti-diagonal
    (r+1,c)-(r,c+1), stored at (r, c); last row and column zero."""
    img = ellipse_image(shape, seed, sigma=sigma)
    w, a = _image_to_grid(img, lam, sigma, beta_sigma)
    ld = lam / np.sqrt(2.0)
    dd = np.zeros_like(img)
    ad = np.zeros_like(img)
    dd[:-1, :-1] = ld * np.exp(-((img[1:, 1:] - img[:-1, :-1]) ** 2) / (2.0 * beta_sigma ** 2))
    ad[:-1, :-1] = ld * np.exp(-((img[:-1, 1:] - img[1:, :-1]) ** 2) / (2.0 * beta_sigma ** 2))
    return w, a + [_quantise(dd), _quantise(ad)]


def edit_sequence(shape, seed, frames, frac=0.02, w_max=20, a_max=10):
    """Integer grid edited frame by frame (as in interactive segmentation):
    frame 0 is `iid_grid`, each later frame redraws a fraction `frac` of the
    unaries of the previous one; the edge weights stay.  Returns a list of (w, a)."""
    w, a = iid_grid(shape, seed, w_max, a_max)
    rng = _rng(seed + 1)
    out = [(w, a)]
    for _ in range(1, frames):
        m = rng.random(w.shape) < frac
        w = w.copy()
        w[m] = rng.integers(-w_max, w_max + 1, size=int(m.sum())).astype(np.float32)
        out.append((w, a))
    return out


def ellipse_sequence(shape, seed, frames, speed=2.0, lam=2.0, sigma=0.15, beta_sigma=0.1):
    """Frames of moving ellipses (a video-like sequence of related cut problems):
    every ellipse drifts by a random velocity of `speed` pixels per frame; each
    frame has fresh noise.  Returns a list of (w, a)."""
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    ells = _ellipses(rng, shape)
    vel = []
    for _ in ells:
        ang = rng.uniform(0, 2 * np.pi)
        vel.append(speed * np.array([np.sin(ang), np.cos(ang)]))
    out = []
    for t in range(frames):
        moved = [(c + t * v, semi, rot) for (c, semi, rot), v in zip(ells, vel)]
        out.append(_image_to_grid(_render(shape, moved, rng, sigma), lam, sigma, beta_sigma))
    return out


def stereo_labels(shape, seed, n_labels=16, sigma=1.2, outliers=0.1, t_data=8, lam_hi=3, lam_lo=1,
                  k_range=(6, 12)):
    """Multi-label problem on an (H, W) grid: (data [L][H][W], [lam_x, lam_y],
    true labels).  Integer values, so every energy is exact; lam_x's last
    column and lam_y's last row are zero."""
    rng = _rng(seed)
    H, W = (int(s) for s in shape)
    L = int(n_labels)
    # background: a plane tilted along W, objects at constant labels on top
    lo, hi = sorted(rng.integers(0, max(1, L // 2), size=2))
    true = np.broadcast_to(np.floor(np.linspace(lo, hi + 0.999, W)), (H, W)).astype(np.int64).copy()
    grids = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    coords = np.stack([g.ravel() for g in grids], axis=1)
    for centre, semi, rot in _ellipses(rng, (H, W), k_range):
        d = (coords - centre) @ rot
        inside = (np.sum((d / semi) ** 2, axis=1) <= 1.0).reshape(H, W)
        true[inside] = int(rng.integers(0, L))
    # observed labels: noise, then outliers anywhere in the label range
    obs = np.rint(true + rng.normal(0.0, sigma, size=(H, W)))
    out = rng.uniform(size=(H, W)) < outliers
    obs[out] = rng.integers(0, L, size=int(out.sum()))
    labels = np.arange(L, dtype=np.float64)[:, None, None]
    data = np.minimum(np.abs(obs[None] - labels), t_data).astype(np.float32)
    # an intensity image with edges where the labels change sets the weights
    img = 8.0 * true + rng.normal(0.0, 2.0, size=(H, W))
    lam_x = np.where(np.abs(np.diff(img, axis=1)) <= 6.0, lam_hi, lam_lo).astype(np.float32)
    lam_y = np.where(np.abs(np.diff(img, axis=0)) <= 6.0, lam_hi, lam_lo).astype(np.float32)
    lx = np.zeros((H, W), np.float32)
    ly = np.zeros((H, W), np.float32)
    lx[:, :-1] = lam_x
    ly[:-1, :] = lam_y
    return data, [lx, ly], true.astype(np.int32)


def batch_sizes(count, seed, lo=128, hi=1024):
    """`count` (H, W) pairs, each dimension uniform on [lo, hi]."""
    rng = _rng(seed)
    return [tuple(int(v) for v in rng.integers(lo, hi + 1, size=2)) for _ in range(count)]


# Named workloads ----------------------------------------------------------

def config_small(seed=1000):
    """64x64 4-connected grid, integer data."""
    return iid_grid((64, 64), seed)


def config_image2d(seed=2000, shape=(1024, 1024)):
    """1024x1024 segmentation-shaped grid, lambda = 2."""
    return ellipse_grid(shape, seed, lam=2.0)


def config_volume3d(seed=3000, shape=(128, 256, 256)):
    """256x256x128 (W x H x D) 6-connected volume, lambda = 1.5."""
    return ellipse_grid(shape, seed, lam=1.5)


def config_batch(seed=4000, count=64):
    """64 uneven integer grids: list of (w, a)."""
    sizes = batch_sizes(count, seed)
    return [iid_grid(hw, seed + 1 + g) for g, hw in enumerate(sizes)]


def config_warm(seed, shape=(512, 512)):
    """512x512 integer grid for the learned warm start."""
    return iid_grid(shape, seed)


# Warm-start network ---------------------------------------------------------

NET_LAYERS = ((3, 32), (32, 32), (32, 32), (32, 2))


def net_init(seed):
    """Seeded He-normal initial parameters of the 4-layer 3x3 network, biases 0.

    Flat float32 vector: for each layer W (index order co, ky, kx, ci), then b."""
    rng = _rng(seed)
    parts = []
    for ci, co in NET_LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=co * 9 * ci))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
