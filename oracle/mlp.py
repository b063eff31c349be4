"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

4 -> 64 -> 64 -> 64 -> 1 with ReLU hidden activations, parameters in the
order W1[64][4], b1, W2[64][64], b2, W3[64][64], b3, W4[64], b4; loss the mean
relative squared error over samples with target w > 0.  Written out layer by
layer in numpy float64, forward and backward by the chain rule.

bf16=True evaluates the network under the surrogate's BF16 rounding rule (a
design choice stated on its own here; the paper has no network): the
weights of the two 64 x 64 layers and the inputs of those layers and of the
output layer (the ReLU outputs of layers 1, 2 and 3) are rounded to BF16
(8 significant bits, round to nearest, ties to even); layer 1's weights and
inputs, the output layer's weights and every bias stay unrounded.  The
gradient treats each rounding as the identity (straight-through): it is the
exact gradient of the same network with the rounding offsets frozen at their
current values.  A change to which tensors are rounded is a change of that
rule, made in its statement first and then here and in the kernels.
"""

from __future__ import annotations

import numpy as np

H, IN = 64, 4
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
         ("W4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = theta[off:off + size].reshape(shape)
        off += size
    return out


def round_bf16(v):
    """Nearest value with 8 significant bits (ties to even), from the
    definition: v = m 2^e with 0.5 <= |m| < 1, round m 2^8 to an integer."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def forward(theta, x, bf16=False):
    p = unpack(theta)
    rnd = round_bf16 if bf16 else (lambda v: v)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ rnd(p["W2"]).T + p["b2"]
    h2 = rnd(np.maximum(z2, 0.0))
    z3 = h2 @ rnd(p["W3"]).T + p["b3"]
    h3 = rnd(np.maximum(z3, 0.0))
    y = h3 @ p["W4"] + p["b4"][0]
    return y, (x, z1, h1, z2, h2, z3, h3)


def loss(theta, x, w, bf16=False):
    y, _ = forward(theta, x, bf16)
    w = np.asarray(w, dtype=np.float64)
    use = w > 0
    r = np.where(use, (y - w) / np.where(use, w, 1.0), 0.0)
    return float(np.sum(r * r) / len(w))


def grad(theta, x, w, bf16=False):
    """Gradient of loss() with respect to theta (same layout); with bf16, the
    straight-through gradient described above."""
    p = unpack(theta)
    y, (x, z1, h1, z2, h2, z3, h3) = forward(theta, x, bf16)
    W2 = round_bf16(p["W2"]) if bf16 else p["W2"]
    W3 = round_bf16(p["W3"]) if bf16 else p["W3"]
    w = np.asarray(w, dtype=np.float64)
    n = len(w)
    use = w > 0
    ws = np.where(use, w, 1.0)
    dy = np.where(use, 2.0 * (y - w) / (ws * ws) / n, 0.0)
    g = {"W4": h3.T @ dy, "b4": np.array([dy.sum()])}
    dz3 = np.outer(dy, p["W4"]) * (z3 > 0)
    g["W3"] = dz3.T @ h2
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ W3) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return np.concatenate([g[name].ravel() for name, _ in SIZES])
