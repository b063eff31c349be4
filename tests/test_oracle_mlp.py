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


def test_round_bf16_matches_library_conversion():
    """The BF16 rounding written from its definition equals torch's
    float32 -> bfloat16 conversion (round to nearest even), including exact
    ties and values across many binades."""
    import torch
    rng = np.random.default_rng(5)
    v = (rng.normal(size=20000) * np.exp2(rng.integers(-40, 40, size=20000))).astype(np.float32)
    bits = rng.integers(0, 2 ** 31, size=4000, dtype=np.int64).astype(np.uint32)
    ties = ((bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)  # exactly halfway
    ties = ties[np.isfinite(ties) & (np.abs(ties) > 1e-30)]
    for arr in (v, ties, -ties):
        ref = torch.from_numpy(arr).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(mlp.round_bf16(arr.astype(np.float64)), ref)


def _frozen_loss(th, x, w, th0):
    """The network with the BF16 rounding offsets frozen at their values for
    th0: W -> W + (round(W0) - W0), h -> h + (round(h0) - h0) for W2, W3 and
    the three hidden layers' outputs."""
    p, p0 = mlp.unpack(th), mlp.unpack(th0)
    dW2 = mlp.round_bf16(p0["W2"]) - p0["W2"]
    dW3 = mlp.round_bf16(p0["W3"]) - p0["W3"]
    h1_0 = np.maximum(x @ p0["W1"].T + p0["b1"], 0.0)
    dh1 = mlp.round_bf16(h1_0) - h1_0
    h2_0 = np.maximum((h1_0 + dh1) @ (p0["W2"] + dW2).T + p0["b2"], 0.0)
    dh2 = mlp.round_bf16(h2_0) - h2_0
    h3_0 = np.maximum((h2_0 + dh2) @ (p0["W3"] + dW3).T + p0["b3"], 0.0)
    dh3 = mlp.round_bf16(h3_0) - h3_0
    h1 = np.maximum(x @ p["W1"].T + p["b1"], 0.0) + dh1
    h2 = np.maximum(h1 @ (p["W2"] + dW2).T + p["b2"], 0.0) + dh2
    h3 = np.maximum(h2 @ (p["W3"] + dW3).T + p["b3"], 0.0) + dh3
    y = h3 @ p["W4"] + p["b4"][0]
    r = np.where(w > 0, (y - w) / np.where(w > 0, w, 1.0), 0.0)
    return float(np.sum(r * r) / len(w))


def test_bf16_gradient_is_straight_through():
    """With bf16=True the oracle's gradient is the exact gradient of the
    network whose rounding offsets are frozen (central differences), and the
    loss at th0 is that network's loss."""
    rng = np.random.default_rng(6)
    th = _theta(7)
    x = rng.normal(size=(24, 4))
    w = rng.uniform(0.5, 2.0, size=24)
    w[5] = 0.0
    assert np.isclose(mlp.loss(th, x, w, bf16=True), _frozen_loss(th, x, w, th), rtol=1e-13)
    g = mlp.grad(th, x, w, bf16=True)
    eps = 1e-6
    for j in rng.choice(mlp.NPARAM, size=60, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[j] += eps
        tm[j] -= eps
        fd = (_frozen_loss(tp, x, w, th) - _frozen_loss(tm, x, w, th)) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-8


def test_bf16_forward_is_close_to_exact():
    """BF16 rounding of two layers' weights and inputs moves the output by a
    few units of 2^-8 relative at most on a random network."""
    rng = np.random.default_rng(8)
    th = _theta(9)
    x = rng.normal(size=(200, 4))
    y, _ = mlp.forward(th, x)
    yb, _ = mlp.forward(th, x, bf16=True)
    assert not np.array_equal(y, yb)
    assert np.max(np.abs(yb - y)) <= 8 * 2.0 ** -8 * np.max(np.abs(y))
