"""Flat LCDM cosmology and the BBKS linear power spectrum used for the inputs.

Readings (the paper runs PINOCCHIO on its own parameter files and does not
state a spectrum): BBKS transfer function with shape parameter
Gamma = Omega_m * h, h = 0.7, no baryon correction; P(k) = A k^n_s T(k)^2 with A
fixed by sigma_8 for a real-space top-hat of radius 8 Mpc/h.  Units: k in
h/Mpc, lengths in Mpc/h.
"""

from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np

H_LITTLE = 0.7


def bbks_transfer(k, omega_m: float, h: float = H_LITTLE):
    """BBKS (1986) fitting formula, q = k / (Omega_m h)."""
    k = np.asarray(k, dtype=np.float64)
    q = k / (omega_m * h)
    out = np.ones_like(q)
    nz = q > 0
    qq = q[nz]
    out[nz] = (np.log1p(2.34 * qq) / (2.34 * qq)
               * (1.0 + 3.89 * qq + (16.1 * qq) ** 2 + (5.46 * qq) ** 3 + (6.71 * qq) ** 4) ** -0.25)
    return out


def _tophat_window(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    big = x > 1e-3
    xb = x[big]
    out[big] = 3.0 * (np.sin(xb) - xb * np.cos(xb)) / xb ** 3
    xs = x[~big]
    out[~big] = 1.0 - xs ** 2 / 10.0 + xs ** 4 / 280.0
    return out


def _simpson_lnk(f_of_k, kmin=1e-6, kmax=1e4, npts=(1 << 16) + 1):
    """Integral of f(k) d ln k by composite Simpson on a uniform ln k grid."""
    lnk = np.linspace(np.log(kmin), np.log(kmax), npts)
    k = np.exp(lnk)
    f = f_of_k(k)
    h = lnk[1] - lnk[0]
    return h / 3.0 * (f[0] + f[-1] + 4.0 * f[1:-1:2].sum() + 2.0 * f[2:-1:2].sum())


def _pk_shape(k, omega_m, n_s, h=H_LITTLE):
    k = np.asarray(k, dtype=np.float64)
    return k ** n_s * bbks_transfer(k, omega_m, h) ** 2


def sigma_tophat(R: float, amplitude: float, omega_m: float, n_s: float, h: float = H_LITTLE):
    """rms of the linear field in a top-hat sphere of radius R."""
    var = _simpson_lnk(lambda k: k ** 3 * amplitude * _pk_shape(k, omega_m, n_s, h)
                       * _tophat_window(k * R) ** 2 / (2.0 * np.pi ** 2))
    return float(np.sqrt(var))


def sigma_gauss(R: float, amplitude: float, omega_m: float, n_s: float, h: float = H_LITTLE):
    """rms of the linear field smoothed with a Gaussian of radius R (continuum)."""
    var = _simpson_lnk(lambda k: k ** 3 * amplitude * _pk_shape(k, omega_m, n_s, h)
                       * np.exp(-(k * R) ** 2) / (2.0 * np.pi ** 2))
    return float(np.sqrt(var))


@dataclass(frozen=True)
class Cosmology:
    omega_m: float = 0.3
    sigma8: float = 0.8
    n_s: float = 0.96
    h: float = H_LITTLE

    @property
    def amplitude(self) -> float:
        return _amplitude(self.omega_m, self.sigma8, self.n_s, self.h)

    def pk(self, k):
        return power_spectrum(k, self)


@lru_cache(maxsize=256)
def _amplitude(omega_m, sigma8, n_s, h):
    unit = sigma_tophat(8.0, 1.0, omega_m, n_s, h)
    return sigma8 ** 2 / unit ** 2


def power_spectrum(k, cosmo: Cosmology):
    """P(k) in (Mpc/h)^3, normalised to cosmo.sigma8."""
    return cosmo.amplitude * _pk_shape(k, cosmo.omega_m, cosmo.n_s, cosmo.h)


def power_spectrum_torch(k, cosmo: Cosmology):
    """The same P(k) on a torch tensor (float64, any device)."""
    import torch
    q = k / (cosmo.omega_m * cosmo.h)
    qs = torch.where(q > 0, q, torch.ones_like(q))
    t = (torch.log1p(2.34 * qs) / (2.34 * qs)
         * (1.0 + 3.89 * qs + (16.1 * qs) ** 2 + (5.46 * qs) ** 3 + (6.71 * qs) ** 4) ** -0.25)
    t = torch.where(q > 0, t, torch.ones_like(t))
    return cosmo.amplitude * torch.where(k > 0, k, torch.ones_like(k)) ** cosmo.n_s * t * t * (k > 0)
