"""Pins of the FP64 warm-start network reference against library routines,
finite differences, adjoint identities and closed forms."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import oracle
from oracle import convnet as cn
from paper_1503_01563_amd import gen


def rng(seed=0):
    return np.random.default_rng(seed)


def test_param_count_and_layout():
    assert cn.param_count() == 864 + 32 + 9216 + 32 + 9216 + 32 + 576 + 2
    p = np.arange(cn.param_count(), dtype=np.float64)
    layers = cn.unpack(p)
    assert layers[0][0].shape == (32, 3, 3, 3) and layers[3][0].shape == (2, 3, 3, 32)
    # W[co, ky, kx, ci] is at offset ((co*3 + ky)*3 + kx)*ci_count + ci
    assert layers[1][0][5, 2, 1, 7] == 864 + 32 + ((5 * 3 + 2) * 3 + 1) * 32 + 7
    np.testing.assert_array_equal(cn.pack(layers), p)
    assert gen.net_init(3).size == cn.param_count()


def test_conv_single_channel_is_library_correlation():
    r = rng(1)
    x = r.normal(size=(9, 13, 1))
    W = r.normal(size=(1, 3, 3, 1))
    out = cn.conv3x3(x, W, np.array([0.25]))
    ref = correlate2d(x[:, :, 0], W[0, :, :, 0], mode="same", boundary="fill") + 0.25
    np.testing.assert_allclose(out[:, :, 0], ref, rtol=1e-13, atol=1e-13)


def test_conv_multichannel_sums_channel_correlations():
    r = rng(2)
    x = r.normal(size=(7, 6, 4))
    W = r.normal(size=(3, 3, 3, 4))
    out = cn.conv3x3(x, W, np.zeros(3))
    for co in range(3):
        ref = sum(correlate2d(x[:, :, ci], W[co, :, :, ci], mode="same") for ci in range(4))
        np.testing.assert_allclose(out[:, :, co], ref, rtol=1e-12, atol=1e-12)


def test_grad_input_is_adjoint_of_conv():
    r = rng(3)
    x = r.normal(size=(8, 5, 6))
    g = r.normal(size=(8, 5, 4))
    W = r.normal(size=(4, 3, 3, 6))
    lhs = np.sum(cn.conv3x3(x, W, np.zeros(4)) * g)
    rhs = np.sum(x * cn.conv3x3_grad_input(g, W))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_grad_weights_is_adjoint_in_w():
    r = rng(4)
    x = r.normal(size=(6, 7, 3))
    g = r.normal(size=(6, 7, 5))
    W = r.normal(size=(5, 3, 3, 3))
    dW, db = cn.conv3x3_grad_weights(x, g)
    # <conv(x; W, b), g> is linear in (W, b) with gradient (dW, db)
    b = r.normal(size=5)
    val = np.sum(cn.conv3x3(x, W, b) * g)
    assert abs(val - (np.sum(dW * W) + np.sum(db * b))) <= 1e-11 * abs(val)


def _small_batch(seed):
    r = rng(seed)
    batch, targets = [], []
    for shape in [(5, 7), (6, 4)]:
        w = r.integers(-20, 21, size=shape).astype(np.float64)
        ax = r.integers(0, 11, size=shape).astype(np.float64)
        ay = r.integers(0, 11, size=shape).astype(np.float64)
        batch.append((w, ax, ay))
        targets.append(r.normal(size=shape + (2,)))
    return batch, targets


def test_gradient_matches_central_differences():
    batch, targets = _small_batch(5)
    p = gen.net_init(11).astype(np.float64)
    p += rng(6).normal(0, 0.05, size=p.size)  # nonzero biases
    loss, g = cn.loss_and_grad(p, batch, targets)
    r = rng(7)
    offs = np.cumsum([0] + [co * 9 * ci + co for ci, co in cn.LAYERS])
    idx = []
    for l in range(4):
        nw = cn.LAYERS[l][1] * 9 * cn.LAYERS[l][0]
        idx += list(offs[l] + r.choice(nw, 12, replace=False))
        idx += list(offs[l] + nw + r.choice(cn.LAYERS[l][1], 2, replace=False))
    h = 1e-6
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (cn.loss_and_grad(pp, batch, targets)[0] - cn.loss_and_grad(pm, batch, targets)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_loss_is_mean_squared_error():
    batch, targets = _small_batch(8)
    p = gen.net_init(12).astype(np.float64)
    loss, _ = cn.loss_and_grad(p, batch, targets)
    outs = [cn.forward(p, *b) for b in batch]
    ref = np.mean(np.concatenate([((o - t) ** 2).ravel() for o, t in zip(outs, targets)]))
    assert abs(loss - ref) <= 1e-14 * ref


def test_zero_weights_give_bias_output():
    layers = cn.unpack(np.zeros(cn.param_count()))
    layers[3][1][...] = [1.5, -2.0]
    out = cn.forward(cn.pack(layers), np.ones((3, 4)), np.ones((3, 4)), np.ones((3, 4)))
    np.testing.assert_array_equal(out[..., 0], 1.5)
    np.testing.assert_array_equal(out[..., 1], -2.0)


def test_adam_closed_forms():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.zeros(4)
    lr, eps = 0.01, 1e-8
    p1, m1, v1 = cn.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr, eps=eps)
    # first step: bias correction makes the update lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    # constant gradient: every step moves by lr * g / (|g| + eps)
    p2, _, _ = cn.adam_step(p1, g, m1, v1, 2, lr, eps=eps)
    np.testing.assert_allclose(p2 - p1, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)


def test_warm_state_dual_is_in_row_family():
    w, a = gen.iid_grid((9, 11), 77)
    r = rng(9)
    out = r.normal(0, 6, size=(9, 11, 2))
    z = cn.warm_state(out, a[0], 0.0)
    # rows sum to zero and the row prox of a member of K_rows is zero
    np.testing.assert_allclose(z.sum(axis=1), 0, atol=1e-12)
    q, _ = oracle.prox_family(z.shape, 0, z, a[0])
    np.testing.assert_allclose(q, 0, atol=1e-10)
    z2 = cn.warm_state(out, a[0], 2.0)
    np.testing.assert_allclose(z2 - z, 2.0 * out[..., 0], atol=1e-12)


def test_round_bf16():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1.5, 3.0e38, 1e-40], np.float32)
    exp = np.array([1.0, 1.0, 1 + 2 ** -6, -1.5])
    np.testing.assert_array_equal(cn.round_bf16(vals)[:4], exp)
    torch = pytest.importorskip("torch")
    x = rng(10).normal(0, 100, size=2000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cn.round_bf16(x), ref)
