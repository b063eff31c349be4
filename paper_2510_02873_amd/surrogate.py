"""Training of the surrogate network on data the collapse method generates.

Every step runs in the library's kernels: network inputs and targets come
from pino_collapse_features (FP64 eigenvalues and the full collapse solve),
gradients and Adam updates from pino_mlp_train_step.  torch only holds the
device buffers and gathers the random minibatches.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import _abi
from .runner import Collapse


def training_pairs(fields, growth_tables, device=0, per_slab=None, stream=None, method=_abi.PINO_CLASSIC):
    """fields: iterable of (hessian (6, n) tensor on the device, sigma_R,
    cosmology index); returns (x [m][4] float32, w [m] float32) device
    tensors of the particles where the network is consulted (w > 0).  The
    targets solve the collapse condition of `method` (PINO_CLASSIC, or
    PINO_CLASSIC_LCDM with FP64 fields: then they depend on each table's
    omega_m, and so does the network's fourth input)."""
    col = None
    xs, ws = [], []
    for h, sigma, cosmo in fields:
        if col is None:
            prec = _abi.PINO_FP64 if h.dtype == torch.float64 else _abi.PINO_MIXED
            col = Collapse(growth_tables, method=method, precision=prec, device=device)
        n = h.shape[1]
        x = torch.empty((n, 4), dtype=torch.float32, device=h.device)
        w = torch.empty(n, dtype=torch.float32, device=h.device)
        F = torch.empty(1, dtype=torch.float64, device=h.device)
        R = torch.empty(1, dtype=torch.int32, device=h.device)
        item = _abi.make_item(h, F, R, None, radius_index=0, cosmo=cosmo, sigma_R=sigma, n=n)
        _abi.pino_collapse_features(col.ctx, item, x, w,
                                    stream=stream or torch.cuda.current_stream(h.device))
        keep = w > 0
        if per_slab is not None:
            idx = torch.nonzero(keep).squeeze(1)
            if idx.numel() > per_slab:
                g = torch.Generator(device=h.device).manual_seed(int(n + cosmo * 7919 + sigma * 1e6))
                idx = idx[torch.randperm(idx.numel(), device=h.device, generator=g)[:per_slab]]
            xs.append(x[idx])
            ws.append(w[idx])
        else:
            xs.append(x[keep])
            ws.append(w[keep])
    if col is not None:
        col.close()
    return torch.cat(xs), torch.cat(ws)


def train(x, w, steps=8000, batch=8192, lr_max=3e-3, seed=0, device=0, log_every=0, log=print,
          bf16_forward=False):
    """One-cycle Adam training; returns (blob, params, history).  With
    bf16_forward the forward pass rounds as the BF16 inference does
    (pino_mlp_set_bf16_forward)."""
    m = _abi.pino_mlp_create(device, seed)
    if bf16_forward:
        _abi.pino_mlp_set_bf16_forward(m, True)
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    gen = torch.Generator(device=x.device).manual_seed(seed)
    hist = []
    try:
        for k in range(steps):
            # one-cycle schedule: linear warm-up over 10%, cosine decay
            f = k / max(steps - 1, 1)
            lr = lr_max * (f / 0.1 if f < 0.1 else 0.5 * (1 + math.cos(math.pi * (f - 0.1) / 0.9)))
            idx = torch.randint(0, x.shape[0], (batch,), device=x.device, generator=gen)
            xb = x[idx].contiguous()
            wb = w[idx].contiguous()
            _abi.pino_mlp_train_step(m, xb, wb, max(lr, 1e-6), loss)
            if log_every and (k % log_every == 0 or k == steps - 1):
                hist.append((k, float(loss.item())))
                log(f"[train] step {k} lr {lr:.2e} loss {hist[-1][1]:.3e}")
        blob = _abi.pino_mlp_export(m)
        params = _abi.pino_mlp_get_params(m)
    finally:
        _abi.pino_mlp_free(m)
    return blob, params, hist


def constant_blob(value=1.0):
    """Blob of a network that ignores its inputs and predicts w = value
    (value 1: the Zel'dovich guess D = 1/l1) -- the method without a trained
    network, for comparisons."""
    p = np.zeros(_abi.PINO_MLP_PARAMS, dtype=np.float32)
    p[-1] = value
    m = _abi.pino_mlp_create(0, 0)
    try:
        _abi.pino_mlp_set_params(m, p)
        return _abi.pino_mlp_export(m)
    finally:
        _abi.pino_mlp_free(m)
