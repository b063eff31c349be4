"""Pins for the oracle's Classic collapse with flat-LCDM time coefficients
(CPU only).

The LCDM growth of the second- and third-order LPT terms (k2, k3a, k3b: the
ratios to their Einstein-de Sitter values) is computed by the oracle as a
Green's-function quadrature.  It is pinned by
  * Einstein-de Sitter (Omega_m = 1): every ratio is 1;
  * scipy's DOP853 integration of the defining ODEs, written here from the
    perturbation equations (not from the oracle's integral form);
  * the Bouchet et al. (1995) power-law fits Omega_m^-1/143, ^-4/275 and
    ^-269/17875 at a = 1 (fits, so within 2e-3).
The collapse root with these coefficients is pinned by
  * Omega_m = 1: it equals the Einstein-de Sitter Classic root;
  * an independent evaluation of the condition with scipy's natural cubic
    spline of the ODE-integrated ratios: the oracle's root is a zero of it,
    and a dense sign scan finds no earlier one;
  * l1 <= 0 never collapses.
"""

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.interpolate import CubicSpline
from scipy.optimize import brentq

import synth


def _ode_ratios(om, a):
    """k2, k3a, k3b at scale factors a from the growth ODEs in x = ln a:
    D'' + (2 - 1.5 Om(a)) D' - 1.5 Om(a) D = S, with S = 0 (D1),
    -1.5 Om(a) D1^2 (D2), -3 Om(a) D1^3 (D3a), -3 Om(a) D1 (D2 - D1^2) (D3b),
    started in the Einstein-de Sitter growing modes at a = 1e-8."""
    def rhs(x, y):
        aa = np.exp(x)
        om_a = om * aa ** -3 / (om * aa ** -3 + 1 - om)
        d1, v1, d2, v2, d3a, v3a, d3b, v3b = y
        p = 2 - 1.5 * om_a
        lin = lambda d, v: -p * v + 1.5 * om_a * d
        return [v1, lin(d1, v1), v2, lin(d2, v2) - 1.5 * om_a * d1 ** 2, v3a, lin(d3a, v3a) - 3 * om_a * d1 ** 3,
                v3b, lin(d3b, v3b) - 3 * om_a * d1 * (d2 - d1 ** 2)]
    a0 = 1e-8
    y0 = [a0, a0, -3 / 7 * a0 ** 2, -6 / 7 * a0 ** 2, -1 / 3 * a0 ** 3, -a0 ** 3, 10 / 21 * a0 ** 3, 10 / 7 * a0 ** 3]
    sol = solve_ivp(rhs, [np.log(a0), np.log(a[-1])], y0, t_eval=np.log(a), rtol=1e-13, atol=1e-60,
                    method="DOP853")
    d1, d2, d3a, d3b = sol.y[0], sol.y[2], sol.y[4], sol.y[6]
    return d2 / (-3 / 7 * d1 ** 2), d3a / (-1 / 3 * d1 ** 3), d3b / (10 / 21 * d1 ** 3)


def test_lpt_growth_eds_is_one(orc):
    a, _ = synth.growth_table(1.0)
    for k in orc.lpt_growth(1.0, a):
        assert np.max(np.abs(k - 1.0)) < 1e-10


@pytest.mark.parametrize("om", [0.25, 0.3, 0.35])
def test_lpt_growth_vs_ode(orc, om):
    a, _ = synth.growth_table(om)
    got = orc.lpt_growth(om, a)
    ref = _ode_ratios(om, a)
    for g, r in zip(got, ref):
        assert np.max(np.abs(g - r)) < 1e-9
    # irregular knots (every knot is a node of the oracle's grid)
    rng = np.random.default_rng(3)
    a2 = np.sort(np.concatenate([[1e-3, 1.0], rng.uniform(1e-3, 1.0, 40)]))
    for g, r in zip(orc.lpt_growth(om, a2), _ode_ratios(om, a2)):
        assert np.max(np.abs(g - r)) < 1e-9


def test_lpt_growth_vs_bouchet_fits(orc):
    for om in (0.25, 0.3, 0.35):
        k2, k3a, k3b = (k[-1] for k in orc.lpt_growth(om, np.array([1e-3, 0.1, 1.0])))
        assert abs(k2 - om ** (-1 / 143)) < 2e-3
        assert abs(k3a - om ** (-4 / 275)) < 2e-3
        assert abs(k3b - om ** (-269 / 17875)) < 2e-3
        # Lambda slows the growth of the linear mode more than that of the
        # higher orders: every ratio exceeds 1 and grows with time
        for k in orc.lpt_growth(om, np.array([1e-2, 0.1, 0.5, 1.0])):
            assert np.all(np.diff(k) > 0) and k[0] > 1.0


def _random_lams(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    lam = -np.sort(-rng.normal(size=(n, 3)) * scale, axis=1)
    return lam


def test_lcdm_collapse_eds_equals_classic(orc):
    a, D = synth.growth_table(1.0)
    g = orc.Growth(a, D, 1.0)
    for lam in _random_lams(300, 5, 1.5):
        d0 = orc.collapse_D(lam)
        d1 = orc.collapse_D_lcdm(lam, g)
        assert (d0 is None) == (d1 is None)
        if d0 is not None:
            assert abs(d1 - d0) <= 1e-9 * d0


def test_lcdm_collapse_root_independent(orc):
    om = 0.3
    a, D = synth.growth_table(om)
    g = orc.Growth(a, D, om)
    ks = [CubicSpline(D, k, bc_type="natural") for k in _ode_ratios(om, a)]

    def G(lam, d):
        b, c = orc.lpt_axis(lam, 0)
        ga = lam[0] * lam[1] * lam[2] / 9.0
        kk = [float(s(min(max(d, D[0]), D[-1]))) for s in ks]
        return 1 - lam[0] * d + kk[0] * b * d * d + (kk[1] * ga + kk[2] * (c - ga)) * d ** 3

    found = 0
    for lam in _random_lams(60, 9, 2.0):
        dc = orc.collapse_D_lcdm(lam, g)
        if lam[0] <= 0:
            assert dc is None
            continue
        if dc is None:
            continue
        found += 1
        # a zero of the independently built condition, within its rounding
        lo, hi = dc * (1 - 1e-8), dc * (1 + 1e-8)
        if G(lam, lo) > 0 > G(lam, hi):
            r = brentq(lambda x: G(lam, x), lo, hi, xtol=1e-15 * dc)
            assert abs(r - dc) <= 1e-9 * dc
        else:
            assert abs(G(lam, dc)) < 1e-9
        # no earlier crossing on a dense scan
        xs = np.linspace(0, dc * (1 - 1e-6), 4001)[1:]
        assert all(G(lam, x) > 0 for x in xs[::10])
    assert found > 20


def test_lcdm_no_collapse_for_nonpositive_l1(orc):
    a, D = synth.growth_table(0.3)
    g = orc.Growth(a, D, 0.3)
    rng = np.random.default_rng(21)
    for _ in range(200):
        lam = -np.sort(-(-np.abs(rng.normal(size=3)) * rng.uniform(0.1, 5)))
        assert lam[0] <= 0
        assert orc.collapse_D_lcdm(lam, g) is None
