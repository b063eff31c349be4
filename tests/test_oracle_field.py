"""Pins of the oracle's Hessian stage (oracle/field.py) against what the
mathematics fixes without any FFT: the closed-form Hessian of a plane wave
(the Poisson potential of A cos(k0.x) is -A cos(k0.x)/k0^2), linearity over
superposed waves, the trace identity tr H = delta_R, and a field with no
power giving zero."""

import numpy as np
import pytest

from oracle import field as ofield


@pytest.mark.parametrize("n_side,box,mode,R", [
    (16, 100.0, (1, 0, 0), 0.0),
    (16, 100.0, (2, -3, 1), 4.0),
    (17, 60.0, (-4, 5, 7), 1.5),        # odd side, negative components
    (24, 200.0, (3, 3, -3), 10.0),      # diagonal direction
    (12, 50.0, (0, 0, 5), 2.0),         # pure z, largest non-Nyquist kz
])
def test_plane_wave_closed_form(n_side, box, mode, R):
    x = np.arange(n_side) * (box / n_side)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    k0 = 2 * np.pi / box * np.asarray(mode, dtype=float)
    amp = 0.7
    delta = amp * np.cos(k0[0] * X + k0[1] * Y + k0[2] * Z)
    got = ofield.hessian(np.fft.rfftn(delta), n_side, box, R)
    want = ofield.plane_wave_hessian(n_side, box, mode, R, amp)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-12 * scale
    # the six components are not interchangeable: a swapped pair would fail
    if len(set(np.abs(mode))) == 3 and 0 not in mode:
        for c in range(3, 6):
            assert np.max(np.abs(want[c] - want[(c + 1 - 3) % 3 + 3])) > 1e-3 * scale


def test_superposition_and_trace():
    n, box, R = 20, 80.0, 3.0
    rng = np.random.default_rng(5)
    modes = [tuple(rng.integers(-9, 10, size=3)) for _ in range(4)]
    modes = [m for m in modes if any(m)]
    amps = rng.uniform(0.2, 1.0, size=len(modes))
    x = np.arange(n) * (box / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    delta = np.zeros((n, n, n))
    want = np.zeros((6, n ** 3))
    for m, a in zip(modes, amps):
        k0 = 2 * np.pi / box * np.asarray(m, dtype=float)
        delta += a * np.cos(k0[0] * X + k0[1] * Y + k0[2] * Z)
        want += ofield.plane_wave_hessian(n, box, m, R, a)
    got = ofield.hessian(np.fft.rfftn(delta), n, box, R)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # tr H = the smoothed density, written out per mode without an FFT
    dR = np.zeros(n ** 3)
    for m, a in zip(modes, amps):
        k0 = 2 * np.pi / box * np.asarray(m, dtype=float)
        dR += a * np.exp(-0.5 * (k0 @ k0) * R * R) * np.cos(k0[0] * X + k0[1] * Y + k0[2] * Z).reshape(-1)
    assert np.max(np.abs(got[0] + got[1] + got[2] - dR)) <= 1e-12 * np.max(np.abs(dR))


def test_constant_field_has_no_hessian():
    n = 10
    delta_k = np.fft.rfftn(np.full((n, n, n), 3.0))
    assert np.max(np.abs(ofield.hessian(delta_k, n, 50.0, 2.0))) <= 1e-15


def test_nyquist_waves_are_dropped():
    """A wave at the Nyquist index of an even side has no defined derivative
    on the grid (+n/2 and -n/2 alias); the stage drops it, and keeps the
    neighbouring modes."""
    n, box = 12, 60.0
    x = np.arange(n) * (box / n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    kn = np.pi / (box / n)                       # Nyquist wavenumber
    k1 = 2 * np.pi / box
    nyq = np.cos(kn * X + k1 * Y) + np.cos(k1 * X + kn * Z)
    # (only the forward transform's rounding leaks into kept modes)
    assert np.max(np.abs(ofield.hessian(np.fft.rfftn(nyq), n, box, 1.0))) <= 1e-13
    mode = (n // 2 - 1, 2, -1)
    k0 = k1 * np.asarray(mode, dtype=float)
    wave = np.cos(k0[0] * X + k0[1] * Y + k0[2] * Z)
    got = ofield.hessian(np.fft.rfftn(wave + nyq), n, box, 1.0)
    want = ofield.plane_wave_hessian(n, box, mode, 1.0)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
