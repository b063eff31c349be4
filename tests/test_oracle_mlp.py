"""Pins of the FP64 reference network used to check the surrogate's
training kernels: central finite differences of the loss, a network whose
output has a closed form, and the masking of samples without a target."""

import numpy as np

import oracle.mlp as mlp


def _theta(seed, scale=0.3):
    return np.random.default_rng(seed).normal(size=mlp.NPARAM) * scale


def test_closed_form_path():
    th = np.zeros(mlp.NPARAM)
    p = mlp.unpack(th)            # views into th
    p["W1"][0, 0] = 1.0
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["W4"][0] = 2.0
    p["b4"][0] = 0.5
    x = np.array([[1.5, 9, 9, 9], [-2.0, 1, 1, 1], [0.25, 0, 0, 0]])
    y, _ = mlp.forward(th, x)
    assert np.allclose(y, 2.0 * np.maximum(x[:, 0], 0.0) + 0.5, rtol=0, atol=1e-15)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    th = _theta(2)
    x = rng.normal(size=(16, 4))
    w = rng.uniform(0.5, 2.0, size=16)
    w[3] = 0.0                                     # ignored sample
    g = mlp.grad(th, x, w)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    eps = 1e-6
    for j in idx:
        tp, tm = th.copy(), th.copy()
        tp[j] += eps
        tm[j] -= eps
        fd = (mlp.loss(tp, x, w) - mlp.loss(tm, x, w)) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-8


def test_samples_without_target_do_not_count():
    rng = np.random.default_rng(3)
    th = _theta(4)
    x = rng.normal(size=(10, 4))
    w = rng.uniform(0.5, 2.0, size=10)
    w0 = w.copy()
    w0[:4] = 0.0
    # loss over n = 10 with 4 ignored equals the 6-sample loss scaled by 6/10
    assert np.isclose(mlp.loss(th, x, w0), mlp.loss(th, x[4:], w[4:]) * 6 / 10)
    assert np.allclose(mlp.grad(th, x, w0), mlp.grad(th, x[4:], w[4:]) * 6 / 10)
