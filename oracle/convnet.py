"""Plain FP64 reference of the warm-start network (test infrastructure only).

Nothing in the GPU library calls this module; it exists so the tests can
check the HIP network kernels against an obviously correct implementation.

The network maps the cut problem (w, a_x, a_y) of a 2D grid to a guess of the
solution of (TV) and of its row-family dual (the learned warm start of the
splitting state; reusing a good starting state is the warm start the paper
describes for DR in Sec. 4.4 and 6.1):

  features  f = (w / 20, a_x / 10, a_y / 10)           3 channels per pixel
  layer l   h_l = relu(conv3x3(h_{l-1}, W_l) + b_l)     l = 1, 2, 3 (32 channels)
  output    o = conv3x3(h_3, W_4) + b_4                 2 channels: x0, p1

conv3x3 is a cross-correlation with zero padding ("same" size):
  out[y, x, co] = b[co] + sum_{ky, kx, ci} W[co, ky, kx, ci] in[y + ky - 1, x + kx - 1, ci]

Parameters are one flat vector: for each layer W_l (index order co, ky, kx, ci)
then b_l.  Loss: mean squared error over all output elements,
L = sum (o - t)^2 / count.  Optimiser: Adam with bias correction.

Arrays are laid out [H][W][C] per image (pixel-major, channels last) and a
batch is a list / leading axis of images.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((3, 32), (32, 32), (32, 32), (32, 2))
W_SCALE = 20.0
A_SCALE = 10.0


def param_count() -> int:
    return sum(co * 9 * ci + co for ci, co in LAYERS)


def unpack(params):
    """Flat vector -> list of (W [co, 3, 3, ci], b [co]) views."""
    params = np.asarray(params, np.float64)
    out, off = [], 0
    for ci, co in LAYERS:
        nw = co * 9 * ci
        W = params[off:off + nw].reshape(co, 3, 3, ci)
        off += nw
        b = params[off:off + co]
        off += co
        out.append((W, b))
    assert off == params.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def features(w, a_x, a_y):
    return np.stack([np.asarray(w, np.float64) / W_SCALE, np.asarray(a_x, np.float64) / A_SCALE,
                     np.asarray(a_y, np.float64) / A_SCALE], axis=-1)


def _pad(x):
    return np.pad(x, ((1, 1), (1, 1), (0, 0)))


def conv3x3(x, W, b):
    """Cross-correlation with zero padding; x [H][W][ci], W [co][3][3][ci]."""
    H, Wd, _ = x.shape
    xp = _pad(x)
    out = np.broadcast_to(b, (H, Wd, W.shape[0])).copy()
    for ky in range(3):
        for kx in range(3):
            out += xp[ky:ky + H, kx:kx + Wd, :] @ W[:, ky, kx, :].T
    return out


def conv3x3_grad_input(g, W):
    """d(loss)/d(in) given g = d(loss)/d(out): in[y, x, ci] receives
    W[co, ky, kx, ci] g[y - ky + 1, x - kx + 1, co]."""
    H, Wd, _ = g.shape
    din = np.zeros((H + 2, Wd + 2, W.shape[3]))
    for ky in range(3):
        for kx in range(3):
            din[ky:ky + H, kx:kx + Wd, :] += g @ W[:, ky, kx, :]
    return din[1:-1, 1:-1, :]


def conv3x3_grad_weights(x, g):
    """d(loss)/dW [co][3][3][ci] and d(loss)/db [co]."""
    H, Wd, ci = x.shape
    xp = _pad(x)
    co = g.shape[2]
    dW = np.zeros((co, 3, 3, ci))
    gm = g.reshape(-1, co)
    for ky in range(3):
        for kx in range(3):
            dW[:, ky, kx, :] = gm.T @ xp[ky:ky + H, kx:kx + Wd, :].reshape(-1, ci)
    return dW, gm.sum(axis=0)


def forward(params, w, a_x, a_y, keep=False):
    """Output [H][W][2] of one image (and the activations when keep)."""
    layers = unpack(params)
    h = features(w, a_x, a_y)
    acts = [h]
    for l, (W, b) in enumerate(layers):
        h = conv3x3(h, W, b)
        if l < len(layers) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return (h, acts) if keep else h


def loss_and_grad(params, batch, targets):
    """MSE loss over a batch and its gradient w.r.t. the flat parameters.

    batch: list of (w, a_x, a_y); targets: list of [H][W][2] arrays."""
    layers = unpack(params)
    count = sum(t.size for t in targets)
    loss = 0.0
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    for (w, ax, ay), t in zip(batch, targets):
        out, acts = forward(params, w, ax, ay, keep=True)
        diff = out - t
        loss += float(np.sum(diff * diff))
        g = 2.0 * diff / count
        for l in range(len(layers) - 1, -1, -1):
            W, _ = layers[l]
            dW, db = conv3x3_grad_weights(acts[l], g)
            grads[l][0][...] += dW
            grads[l][1][...] += db
            if l > 0:
                g = conv3x3_grad_input(g, W) * (acts[l] > 0)
    return loss / count, pack(grads)


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def warm_state(out, a_x, c):
    """Starting state of the two-set splitting from a network output:
    z0 = c x0 + D_rows^T clip(p1, -a_x, a_x), (D^T p)_i = p_{i-1} - p_i."""
    x0 = np.asarray(out[..., 0], np.float64)
    p = np.clip(np.asarray(out[..., 1], np.float64), -np.asarray(a_x, np.float64), np.asarray(a_x, np.float64))
    y = -p.copy()
    y[:, 1:] += p[:, :-1]
    return c * x0 + y


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
