"""Gaussian linear fields and the Hessian of the smoothed potential.

Sec. 3 of the paper: the linear density contrast delta is a Gaussian field on
a uniform periodic grid, related to the potential by the Poisson equation
nabla^2 phi = delta; for each smoothing radius the second derivatives
d_i d_j phi of the smoothed potential are computed with FFTs.  In Fourier
space that is H_ij(k) = (k_i k_j / k^2) delta(k) W(kR) with a Gaussian window
W = exp(-k^2 R^2 / 2), so the trace of H is the smoothed delta (sign reading:
overdense regions have positive eigenvalues).

Conventions (readings):
  * delta(k) = rfftn(w) * sqrt(P(k) / V_cell) with w ~ N(0,1) white noise in
    real space, so <delta^2> = sum_k P(k) / L^3;
  * the k = 0 mode and every mode with any |k_i| at the Nyquist frequency are
    zeroed, which keeps the real inverse transform exactly Hermitian;
  * the field is the linear field at a = 1 (D = 1).

Output layout is structure-of-arrays: one contiguous array per component in
the order xx, yy, zz, xy, xz, yz, particle index i = (ix * n + iy) * n + iz.
"""

from __future__ import annotations

import numpy as np
import torch

from .cosmo import Cosmology, power_spectrum, power_spectrum_torch

HESSIAN_COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def log_radii(r_max: float, r_min: float, count: int):
    """`count` radii log-spaced from r_max down to r_min (processing order)."""
    if count == 1:
        return [float(r_max)]
    return [float(r_max * (r_min / r_max) ** (k / (count - 1))) for k in range(count)]


def white_noise(n_side: int, seed: int) -> np.ndarray:
    """Unit-variance Gaussian white noise on an n^3 grid (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n_side, n_side, n_side), dtype=np.float64)


def _wavenumbers(n_side: int, box: float, device):
    kf = 2.0 * np.pi / box
    k1 = torch.fft.fftfreq(n_side, d=1.0 / n_side, dtype=torch.float64, device=device) * kf
    kz = torch.fft.rfftfreq(n_side, d=1.0 / n_side, dtype=torch.float64, device=device) * kf
    return k1, kz


def _mode_mask(n_side: int, device):
    """1 for kept modes, 0 for k = 0 and Nyquist modes (rfft half-grid)."""
    m1 = torch.ones(n_side, dtype=torch.float64, device=device)
    mz = torch.ones(n_side // 2 + 1, dtype=torch.float64, device=device)
    if n_side % 2 == 0:
        m1[n_side // 2] = 0.0
        mz[n_side // 2] = 0.0
    mask = m1[:, None, None] * m1[None, :, None] * mz[None, None, :]
    mask[0, 0, 0] = 0.0
    return mask


class _Field:
    """delta(k) of one realisation, kept on `device` for repeated smoothing."""

    def __init__(self, n_side: int, box: float, seed: int, cosmo: Cosmology, device):
        self.n = n_side
        self.box = box
        self.device = torch.device(device)
        noise = torch.from_numpy(white_noise(n_side, seed)).to(self.device)
        dk = torch.fft.rfftn(noise)
        del noise
        k1, kz = _wavenumbers(n_side, box, self.device)
        self.kx = k1[:, None, None]
        self.ky = k1[None, :, None]
        self.kz = kz[None, None, :]
        k2 = self.kx ** 2 + self.ky ** 2 + self.kz ** 2
        kmag = torch.sqrt(k2)
        vcell = (box / n_side) ** 3
        pk = power_spectrum_torch(kmag, cosmo)
        amp = torch.sqrt(pk / vcell) * _mode_mask(n_side, self.device)
        self.dk = dk * amp
        self.k2 = torch.where(k2 > 0, k2, torch.ones_like(k2))
        del dk, amp, pk, kmag

    def hessian(self, R: float, dtype=torch.float64, out=None):
        """(6, n^3) SoA tensor of H_ij for smoothing radius R."""
        n = self.n
        if out is None:
            out = torch.empty((6, n ** 3), dtype=dtype, device=self.device)
        smooth = self.dk * torch.exp(-0.5 * self.k2 * R * R)
        kv = (self.kx, self.ky, self.kz)
        for c, (i, j) in enumerate(_PAIRS):
            comp = torch.fft.irfftn(smooth * (kv[i] * kv[j] / self.k2), s=(n, n, n))
            out[c].copy_(comp.reshape(-1))
            del comp
        return out

    def delta(self, R: float):
        """Smoothed density contrast (for tests of the trace)."""
        n = self.n
        return torch.fft.irfftn(self.dk * torch.exp(-0.5 * self.k2 * R * R), s=(n, n, n)).reshape(-1)


def hessian_radius(n_side: int, box: float, R: float, seed: int, cosmo: Cosmology = Cosmology(),
                   device="cpu", dtype=torch.float64):
    """Hessian SoA (6, n^3) of one realisation at one radius."""
    return _Field(n_side, box, seed, cosmo, device).hessian(R, dtype)


def hessian_slabs(n_side: int, box: float, radii, seed: int, cosmo: Cosmology = Cosmology(),
                  device="cpu", dtype=torch.float64):
    """Yield (R, (6, n^3) tensor) for each radius in the given order."""
    field = _Field(n_side, box, seed, cosmo, device)
    for R in radii:
        yield R, field.hessian(R, dtype)


def field(n_side: int, box: float, seed: int, cosmo: Cosmology = Cosmology(), device="cpu"):
    return _Field(n_side, box, seed, cosmo, device)


def grid_sigma_gauss(n_side: int, box: float, R, cosmo: Cosmology = Cosmology(), device=None):
    """Expected rms of the smoothed field on this grid: sqrt(sum_k P W^2 / L^3)
    over the kept modes (full complex grid, so each mode counts once).  R may
    be a number or a sequence (then a list is returned).  With a torch
    `device` the sum runs there over the real-FFT half grid (the kz = 0 plane
    once, the other kept kz planes twice), which is what large grids need."""
    if device is not None:
        return _grid_sigma_gauss_torch(n_side, box, R, cosmo, device)
    radii = np.atleast_1d(np.asarray(R, dtype=np.float64))
    k1 = np.fft.fftfreq(n_side, d=1.0 / n_side) * (2.0 * np.pi / box)
    keep = np.ones(n_side)
    if n_side % 2 == 0:
        keep[n_side // 2] = 0.0
    total = np.zeros(len(radii))
    ky = k1[:, None]
    kz = k1[None, :]
    for ix in range(n_side):
        if keep[ix] == 0.0:
            continue
        k2 = k1[ix] ** 2 + ky ** 2 + kz ** 2
        w = keep[:, None] * keep[None, :]
        if ix == 0:
            w = w.copy()
            w[0, 0] = 0.0
        pk = w * power_spectrum(np.sqrt(k2).ravel(), cosmo).reshape(k2.shape)
        for j, Rj in enumerate(radii):
            total[j] += float(np.sum(pk * np.exp(-k2 * Rj * Rj)))
    out = [float(np.sqrt(t / box ** 3)) for t in total]
    return out if np.ndim(R) else out[0]


def _grid_sigma_gauss_torch(n_side, box, R, cosmo, device):
    radii = np.atleast_1d(np.asarray(R, dtype=np.float64))
    dev = torch.device(device)
    k1, kz = _wavenumbers(n_side, box, dev)
    mask = _mode_mask(n_side, dev)
    wz = torch.full((n_side // 2 + 1,), 2.0, dtype=torch.float64, device=dev)
    wz[0] = 1.0
    weight = mask * wz[None, None, :]
    k2 = k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz[None, None, :] ** 2
    pk = power_spectrum_torch(torch.sqrt(k2), cosmo) * weight
    out = [float(torch.sqrt(torch.sum(pk * torch.exp(-k2 * (Rj * Rj))) / box ** 3)) for Rj in radii]
    return out if np.ndim(R) else out[0]
