"""Checks of the seeded input generator (CPU).

The generator stands in for the upstream stages (Sec. 3): a Gaussian delta
with a CDM spectrum and the FFT Hessian of the smoothed potential.  Checked
against the spectrum normalisation, the trace identity tr H = delta_R, the
one-point covariance of a Gaussian Hessian and the Doroshkevich probability
that all three eigenvalues are negative.
"""

import numpy as np
import pytest
import scipy.integrate

from synth import (Cosmology, bbks_transfer, grid_sigma_gauss, log_radii, sigma_gauss,
                   sigma_tophat)
from synth.fields import field as make_field


def test_sigma8_normalisation():
    c = Cosmology()
    assert sigma_tophat(8.0, c.amplitude, c.omega_m, c.n_s) == pytest.approx(0.8, rel=1e-10)


def test_sigma_gauss_vs_scipy():
    c = Cosmology()
    A = c.amplitude
    for R in (0.5, 2.0, 8.0):
        integrand = lambda lnk: (np.exp(lnk) ** 3 * A * np.exp(lnk) ** c.n_s
                                 * bbks_transfer(np.exp(lnk), c.omega_m) ** 2
                                 * np.exp(-(np.exp(lnk) * R) ** 2) / (2 * np.pi ** 2))
        val, _ = scipy.integrate.quad(integrand, np.log(1e-6), np.log(1e4), limit=500, epsrel=1e-10)
        assert sigma_gauss(R, A, c.omega_m, c.n_s) == pytest.approx(np.sqrt(val), rel=1e-7)


def test_log_radii():
    r = log_radii(20.0, 0.5, 25)
    assert r[0] == 20.0 and abs(r[-1] - 0.5) < 1e-14 and all(a > b for a, b in zip(r, r[1:]))


def test_trace_and_covariance():
    c = Cosmology()
    f = make_field(48, 150.0, 5, c)
    R = 4.0
    h = f.hessian(R).numpy()
    d = f.delta(R).numpy()
    assert np.max(np.abs(h[0] + h[1] + h[2] - d)) < 1e-13
    sig = grid_sigma_gauss(48, 150.0, R, c)
    assert d.std() == pytest.approx(sig, rel=0.1)
    # Gaussian isotropic Hessian: <H_ii^2> = 3 s^2/15, <H_ii H_jj> = s^2/15,
    # <H_ij^2> = s^2/15 (i != j), with s the rms of the trace
    s2 = d.var()
    assert np.mean(h[0] ** 2) == pytest.approx(3 * s2 / 15, rel=0.15)
    assert np.mean(h[0] * h[1]) == pytest.approx(s2 / 15, rel=0.25)
    assert np.mean(h[3] ** 2) == pytest.approx(s2 / 15, rel=0.15)
    assert abs(np.mean(h[3] * h[4])) < 0.1 * s2 / 15


def test_grid_sigma_half_grid_sum_equals_full_grid_sum():
    """The real-FFT half-grid sum (device version) counts every kept mode of
    the full complex grid exactly once, for even and odd sides."""
    c = Cosmology(0.27, 0.85)
    for n, box in ((24, 90.0), (17, 60.0)):
        radii = [0.7, 2.0, 5.0]
        full = grid_sigma_gauss(n, box, radii, c)
        half = grid_sigma_gauss(n, box, radii, c, device="cpu")
        assert half == pytest.approx(full, rel=1e-12)
    assert grid_sigma_gauss(24, 90.0, 2.0, c, device="cpu") == pytest.approx(grid_sigma_gauss(24, 90.0, 2.0, c),
                                                                              rel=1e-12)


def test_doroshkevich_all_negative_fraction():
    f = make_field(64, 200.0, 6, Cosmology())
    h = f.hessian(3.0).numpy()
    H = np.zeros((h.shape[1], 3, 3))
    for c, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        H[:, i, j] = h[c]
        H[:, j, i] = h[c]
    lam = np.linalg.eigvalsh(H)
    # Doroshkevich (1970): P(l1 < 0) = 0.08 for a Gaussian field
    assert (lam[:, 2] < 0).mean() == pytest.approx(0.08, abs=0.01)


def test_seeded_reproducible():
    a = make_field(16, 50.0, 3, Cosmology()).hessian(2.0)
    b = make_field(16, 50.0, 3, Cosmology()).hessian(2.0)
    assert bool((a == b).all())
