"""Oracle of the Hessian stage (TEST INFRASTRUCTURE ONLY): the second
derivatives of the smoothed potential from the linear density field, with
numpy's FFT (pocketfft) in FP64.  Only the test suite and the benchmark's
CPU-baseline leg may use it; it shares no code with the HIP library.

Sec. 3 of the paper: the potential obeys the Poisson equation, here
nabla^2 phi = delta, and for each smoothing radius R the Hessian of the
smoothed potential is built with FFTs.  In Fourier space, with the Gaussian
window W = exp(-k^2 R^2 / 2),

    H_ij(k) = (k_i k_j / k^2) W(kR) delta(k),     H_ij(k = 0) = 0,

so that tr H = delta_R; modes at the Nyquist index of an even side are
dropped (see kept_modes).  delta(k) is the real-FFT half grid of delta(x) on a
periodic n^3 grid of side L (numpy.fft.rfftn convention: forward transform
unnormalised, axes x, y, z with z halved), wavenumbers numpy.fft.fftfreq
(the Nyquist index of an even side carries -n/2) along x and y and
numpy.fft.rfftfreq along z, times 2 pi / L.  The inverse is numpy.fft.irfftn
(normalised by 1/n^3).  Output layout: (6, n^3), components xx, yy, zz, xy,
xz, yz, particle (ix * n + iy) * n + iz.
"""

from __future__ import annotations

import numpy as np

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def wavenumbers(n_side: int, box: float):
    kf = 2.0 * np.pi / box
    k1 = np.fft.fftfreq(n_side, d=1.0 / n_side) * kf
    kz = np.fft.rfftfreq(n_side, d=1.0 / n_side) * kf
    return k1[:, None, None], k1[None, :, None], kz[None, None, :]


def kept_modes(n_side: int):
    """1 where a mode enters the Hessian, 0 at k = 0 and, for an even side, at
    the Nyquist index along any axis (a wave at the Nyquist frequency has no
    defined derivative on the grid: +n/2 and -n/2 alias)."""
    keep1 = np.ones(n_side)
    keepz = np.ones(n_side // 2 + 1)
    if n_side % 2 == 0:
        keep1[n_side // 2] = 0.0
        keepz[n_side // 2] = 0.0
    keep = keep1[:, None, None] * keep1[None, :, None] * keepz[None, None, :]
    keep[0, 0, 0] = 0.0
    return keep


def hessian(delta_k: np.ndarray, n_side: int, box: float, R: float) -> np.ndarray:
    """(6, n^3) FP64 Hessian of the potential smoothed at radius R."""
    kx, ky, kz = wavenumbers(n_side, box)
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    kv = (kx, ky, kz)
    with np.errstate(divide="ignore", invalid="ignore"):
        base = np.where(kept_modes(n_side) > 0, np.exp(-0.5 * k2 * R * R) / k2, 0.0) * delta_k
    out = np.empty((6, n_side ** 3))
    for c, (i, j) in enumerate(PAIRS):
        out[c] = np.fft.irfftn(base * (kv[i] * kv[j]), s=(n_side,) * 3, axes=(0, 1, 2)).reshape(-1)
    return out


def plane_wave_hessian(n_side: int, box: float, mode, R: float, amplitude: float = 1.0) -> np.ndarray:
    """Closed form for delta(x) = A cos(k0 . x), k0 = 2 pi/L * mode: the
    potential is -A cos(k0 . x)/k0^2, so H_ij = A (k0_i k0_j / k0^2)
    cos(k0 . x) exp(-k0^2 R^2 / 2).  No FFT involved."""
    k0 = 2.0 * np.pi / box * np.asarray(mode, dtype=np.float64)
    k02 = float(k0 @ k0)
    x = np.arange(n_side) * (box / n_side)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    phase = np.cos(k0[0] * X + k0[1] * Y + k0[2] * Z).reshape(-1)
    w = amplitude * np.exp(-0.5 * k02 * R * R) / k02
    return np.stack([w * k0[i] * k0[j] * phase for i, j in PAIRS])
