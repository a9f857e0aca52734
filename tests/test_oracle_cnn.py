"""Pins of the CNN oracle (oracle/cnn.py): library routines, finite differences, Adam's known
first step."""
from __future__ import annotations

import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn
import workloads as wl


def test_bf16_matches_torch():
    import torch
    g = np.random.default_rng(0)
    x = np.concatenate([g.normal(size=5000) * 10.0 ** g.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 3.00390625, 3.0117187500001, 65504.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(x), ref)


def test_conv_matches_scipy_correlate():
    g = np.random.default_rng(1)
    X = g.normal(size=(7, 9, 3))
    Wt = g.normal(size=(9, 4, 3))
    b = g.normal(size=4)
    Z = cnn.conv3x3(X, Wt, b)
    for co in range(4):
        ref = np.full(X.shape[:2], b[co])
        for ci in range(3):
            k = Wt[:, co, ci].reshape(3, 3)  # k[dy, dx] applied at offset (dy-1, dx-1)
            ref += ndimage.correlate(X[:, :, ci], k, mode="wrap")
        assert np.allclose(Z[:, :, co], ref, rtol=1e-12, atol=1e-12)


def test_conv_adjoints():
    # <conv(X), Y> = <X, conv^T(Y)> and the weight gradient is d<conv(X),Y>/dW
    g = np.random.default_rng(2)
    X = g.normal(size=(6, 5, 3))
    Y = g.normal(size=(6, 5, 4))
    Wt = g.normal(size=(9, 4, 3))
    z = np.zeros(4)
    lhs = np.sum(cnn.conv3x3(X, Wt, z) * Y)
    assert np.isclose(lhs, np.sum(X * cnn.conv3x3_transpose(Y, Wt)), rtol=1e-12)
    dW = cnn.conv3x3_weight_grad(Y, X)
    assert np.isclose(lhs, np.sum(dW * Wt), rtol=1e-12)


def test_features_interface():
    img = wl.checkerboard(8, 8, 2)
    X0 = cnn.features(img)
    assert np.array_equal(X0[..., 0], img)
    assert X0[..., 1].all()          # every chess pixel touches the other phase
    X0 = cnn.features(wl.stripes(12, 6, 6, 3))
    assert np.array_equal(X0[0, :, 1], np.array([1, 0, 1, 1, 0, 1] * 2))


def test_gradient_finite_differences():
    # float64 mode (no rounding): the backward pass equals central differences of the loss
    imgs = [wl.random_binary(7, 6, 0.5, 3), wl.random_binary(7, 6, 0.4, 4)]
    params = cnn.init_params(5).astype(np.float64)
    p = cnn.unpack(params)
    for k in ("b1", "b2", "b3"):
        p[k] = np.full_like(p[k], 0.05)  # keep units active
    params = np.concatenate([p[k].ravel() for k, _ in cnn.SHAPES])
    g = np.random.default_rng(6)
    samples = np.array([[i % 2, g.integers(42), g.integers(42), g.normal()] for i in range(10)])
    loss, grad = cnn.loss_and_grad(params, imgs, samples, bf16_mode=False)
    idx = g.choice(cnn.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [cnn.N_PARAMS - 1, cnn.N_PARAMS - 2, 0]])
    h = 1e-6
    for i in idx:
        pp = params.copy()
        pp[i] += h
        lp, _ = cnn.loss_and_grad(pp, imgs, samples, bf16_mode=False)
        pp[i] -= 2 * h
        lm, _ = cnn.loss_and_grad(pp, imgs, samples, bf16_mode=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_adam_first_step_is_lr_times_sign():
    # with bias correction the first step of Adam moves every parameter by lr * sign(g)
    # (up to eps), whatever the gradient's scale
    g = np.array([1e-3, -5.0, 2e2, -1e-1], np.float32)
    p, m, v = cnn.adam(np.zeros(4, np.float32), g, np.zeros(4, np.float32), np.zeros(4, np.float32),
                       1, lr=0.01, eps=1e-12)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-5)


def test_adam_minimises_quadratic():
    target = np.array([1.0, -2.0, 0.5], np.float32)
    p = np.zeros(3, np.float32)
    m = np.zeros(3, np.float32)
    v = np.zeros(3, np.float32)
    for t in range(1, 3001):
        p, m, v = cnn.adam(p, 2 * (p - target), m, v, t, lr=0.01)
    assert np.allclose(p, target, atol=1e-3)
