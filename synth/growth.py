"""Linear growth table D(a) on the grid of scale factors.

Sec. 3 of the paper: D(a) is obtained by solving the ODE of linear growth on a
predefined grid and is then inverted with a cubic spline to get a(D).  The
table is an input of the collapse path; this module produces it.

Flat LCDM without radiation, E^2(a) = Omega_m a^-3 + 1 - Omega_m.  With
y = ln a and V = dD/dy the growth equation is

    dD/dy = V,
    dV/dy = -(2 - 1.5 Om(a)) V + 1.5 Om(a) D,   Om(a) = Omega_m a^-3 / E^2,

integrated with classical fourth-order Runge-Kutta from a = 1e-6 with the
growing-mode start D = V = a, then normalised to D(a = 1) = 1.  Reading: the
grid is log-uniform in a (the paper does not state its spacing).

mu0: the modified-gravity option of the ellipsoid tables, the source term
scaled by mu(a) = 1 + mu0 / E(a)^2 (0: general relativity, the default).
"""

from __future__ import annotations

import numpy as np


def _rhs(y, D, V, omega_m, mu0=0.0):
    a3 = np.exp(-3.0 * y)                  # a^-3
    e2 = omega_m * a3 + 1.0 - omega_m
    om = omega_m * a3 / e2
    mu = 1.0 + mu0 / e2
    return V, -(2.0 - 1.5 * om) * V + 1.5 * om * mu * D


def _rk4(y0, y1, D, V, omega_m, steps, mu0=0.0):
    h = (y1 - y0) / steps
    y = y0
    for _ in range(steps):
        k1d, k1v = _rhs(y, D, V, omega_m, mu0)
        k2d, k2v = _rhs(y + 0.5 * h, D + 0.5 * h * k1d, V + 0.5 * h * k1v, omega_m, mu0)
        k3d, k3v = _rhs(y + 0.5 * h, D + 0.5 * h * k2d, V + 0.5 * h * k2v, omega_m, mu0)
        k4d, k4v = _rhs(y + h, D + h * k3d, V + h * k3v, omega_m, mu0)
        D = D + h / 6.0 * (k1d + 2.0 * k2d + 2.0 * k3d + k4d)
        V = V + h / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v)
        y = y + h
    return D, V


def growth_table(omega_m: float, n: int = 512, a_min: float = 1e-3, a_max: float = 1.0,
                 substeps: int = 64, mu0: float = 0.0):
    """Return (a, D) float64 arrays of length n: a log-uniform in [a_min, a_max],
    D(a) normalised so that D(a_max) = 1 when a_max = 1."""
    if n < 4:
        raise ValueError("growth table needs at least 4 points")
    ya = np.linspace(np.log(a_min), np.log(a_max), n)
    a = np.exp(ya)
    a[0], a[-1] = a_min, a_max
    y_start = np.log(1e-6)
    D, V = np.exp(y_start), np.exp(y_start)
    D, V = _rk4(y_start, ya[0], D, V, omega_m, 4000, mu0)
    out = np.empty(n)
    out[0] = D
    for k in range(1, n):
        D, V = _rk4(ya[k - 1], ya[k], D, V, omega_m, substeps, mu0)
        out[k] = D
    # normalise at a = 1 (integrate on if the table stops earlier)
    if a_max < 1.0:
        D1, _ = _rk4(ya[-1], 0.0, D, V, omega_m, 4000, mu0)
    else:
        D1 = out[-1]
    return a, out / D1
