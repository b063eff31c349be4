"""Pins for the oracle's interpolators, growth inversion and max over radii.

Spline (Sec. 4.2, natural cubic as in the library the paper replaces):
exactness on linear data, equality with scipy's natural CubicSpline, and the
paper's own test function y = x^2 on 512 random knots (Sec. 4.3).
Bilinear + delta-spline table (Sec. 3, Sec. 4.3): exactness on data that is
bilinear in (x, y) times linear in delta, agreement with scipy's
RegularGridInterpolator, and the paper's z = x^2 + y^2 on a 64 x 64 grid.
Growth (Sec. 3): D = a exactly for Omega_m = 1, agreement with an
independent quadrature of the growth integral, and the growth tables of the
input generator (Runge-Kutta ODE) against the oracle's closed form.
Max over radii (Sec. 4.1): brute-force argmax, strict ties, NaN inputs.
"""

import numpy as np
import pytest
import scipy.integrate
import scipy.interpolate

from synth import Cosmology, growth_table, hessian_slabs, table_grid_hessians, table_knots


def test_spline_exact_on_linear(orc):
    rng = np.random.default_rng(1)
    x = np.sort(rng.uniform(-3, 5, 64))
    y = 2.5 * x - 0.75
    M = orc.spline_natural(x, y)
    # M vanishes up to the rounding of the divided differences (~eps*slope/h)
    assert np.max(np.abs(M)) < 1e-13 * 2.5 / np.min(np.diff(x)) * 64
    q = rng.uniform(x[0], x[-1], 1000)
    assert np.max(np.abs(orc.spline_eval(x, y, M, q) - (2.5 * q - 0.75))) < 1e-13


def test_spline_matches_scipy_natural(orc):
    rng = np.random.default_rng(2)
    x = np.sort(rng.uniform(0, 10, 512))
    x = np.unique(x)
    y = np.sin(x) + 0.1 * x ** 2
    M = orc.spline_natural(x, y)
    ref = scipy.interpolate.CubicSpline(x, y, bc_type="natural")
    assert np.max(np.abs(M - ref(x, 2))) < 1e-9 * np.max(np.abs(M))
    q = np.concatenate([rng.uniform(x[0], x[-1], 2000), x])
    got = orc.spline_eval(x, y, M, q)
    assert np.max(np.abs(got - ref(q))) < 1e-12


def test_spline_paper_x_squared(orc):
    # Sec. 4.3: y = x^2 on 512 random knots, random queries; the natural end
    # condition makes the end intervals the only visible error
    rng = np.random.default_rng(3)
    x = np.unique(np.sort(rng.uniform(0, 1, 512)))
    y = x ** 2
    M = orc.spline_natural(x, y)
    q = rng.uniform(x[0], x[-1], 20000)
    res = orc.spline_eval(x, y, M, q) - q ** 2
    interior = (q > x[8]) & (q < x[-9])
    assert np.max(np.abs(res[interior])) < 1e-9
    assert np.mean(np.abs(res)) / np.mean(q ** 2) < 1e-5


def test_spline_rejects_bad_knots(orc):
    with pytest.raises(ValueError):
        orc.spline_natural([0.0, 1.0, 1.0], [0, 1, 2])
    with pytest.raises(ValueError):
        orc.spline_natural([0.0], [0.0])


def _table(orc, fn, nx=64, ny=64, nd=128, seed=4):
    rng = np.random.default_rng(seed)
    xk = np.sort(np.concatenate([[0.0, 6.0], rng.uniform(0, 6, nx - 2)]))
    yk = np.sort(np.concatenate([[0.0, 6.0], rng.uniform(0, 6, ny - 2)]))
    dk = np.sort(np.concatenate([[-6.0, 8.0], rng.uniform(-6, 8, nd - 2)]))
    X, Y, Dl = np.meshgrid(xk, yk, dk, indexing="ij")
    F = fn(X, Y, Dl)
    return orc.Table(xk, yk, dk, F)


def _lam_from(delta, x, y):
    return np.array([(delta + 2 * x + y) / 3, (delta - x + y) / 3, (delta - x - 2 * y) / 3])


def test_table_exact_bilinear_times_linear(orc):
    fn = lambda x, y, d: (0.3 + 0.2 * x + 0.1 * y + 0.05 * x * y) * (2.0 + 0.1 * d)
    t = _table(orc, fn)
    rng = np.random.default_rng(5)
    for _ in range(500):
        x, y, d = rng.uniform(0, 6), rng.uniform(0, 6), rng.uniform(-6, 8)
        got = orc.table_F(t.xk, t.yk, t.dk, t.F, t.M, _lam_from(d, x, y))
        assert got == pytest.approx(fn(x, y, d), rel=1e-12, abs=1e-13)


def test_table_matches_regular_grid_interpolator(orc):
    rng = np.random.default_rng(6)
    vals = rng.uniform(0.1, 2.0, size=(64, 64))
    fn = lambda x, y, d: vals[np.searchsorted(xk, x), np.searchsorted(yk, y)] + 0 * d
    xk = np.sort(np.concatenate([[0.0, 6.0], rng.uniform(0, 6, 62)]))
    yk = np.sort(np.concatenate([[0.0, 6.0], rng.uniform(0, 6, 62)]))
    dk = np.linspace(-6, 8, 16)
    F = np.repeat(vals[:, :, None], 16, axis=2)
    t = orc.Table(xk, yk, dk, F)
    ref = scipy.interpolate.RegularGridInterpolator((xk, yk), vals, method="linear")
    for _ in range(500):
        x, y, d = rng.uniform(0, 6), rng.uniform(0, 6), rng.uniform(-6, 8)
        got = orc.table_F(t.xk, t.yk, t.dk, t.F, t.M, _lam_from(d, x, y))
        assert got == pytest.approx(float(ref([x, y])[0]), rel=1e-12)


def test_table_paper_x2_plus_y2(orc):
    # Sec. 4.3: z = x^2 + y^2 on a 64 x 64 grid of random nodes, each with a
    # 128-knot spline; bilinear error is O(h^2), reported as mean relative
    t = _table(orc, lambda x, y, d: x ** 2 + y ** 2 + 0 * d)
    rng = np.random.default_rng(7)
    rel = []
    for _ in range(2000):
        x, y, d = rng.uniform(0.5, 6), rng.uniform(0.5, 6), rng.uniform(-6, 8)
        got = orc.table_F(t.xk, t.yk, t.dk, t.F, t.M, _lam_from(d, x, y))
        rel.append(abs(got - (x * x + y * y)) / (x * x + y * y))
    assert np.mean(rel) < 2e-3


def test_table_clamps_and_nonnegative(orc):
    t = _table(orc, lambda x, y, d: 1.0 - 0.5 * d + 0 * x)
    # far outside the knots: clamped to the corner row, and F is never < 0
    got = orc.table_F(t.xk, t.yk, t.dk, t.F, t.M, _lam_from(100.0, 50.0, 50.0))
    assert got == 0.0
    got = orc.table_F(t.xk, t.yk, t.dk, t.F, t.M, _lam_from(-100.0, -1.0, -1.0))
    assert got == pytest.approx(1.0 + 3.0, rel=1e-12)


def test_growth_eds_is_identity(orc):
    for a in (1e-3, 0.01, 0.3, 1.0):
        assert orc.lib().orc_growth_D(1.0, a) == pytest.approx(a, rel=1e-12)


def test_growth_closed_form_vs_quadrature(orc):
    om = 0.3
    E = lambda a: np.sqrt(om / a ** 3 + 1 - om)
    def D_quad(a):
        val, _ = scipy.integrate.quad(lambda x: 1.0 / (x * E(x)) ** 3, 0, a, epsabs=0, epsrel=1e-13, limit=200)
        return 2.5 * om * E(a) * val
    for a in (1e-3, 0.1, 0.5, 1.0):
        assert orc.lib().orc_growth_unnorm(om, a) == pytest.approx(D_quad(a), rel=1e-11)
    # LCDM suppresses growth relative to EdS: the Carroll-Press-Turner fit
    ol = 1 - om
    cpt = 2.5 * om / (om ** (4 / 7) - ol + (1 + om / 2) * (1 + ol / 70))
    assert orc.lib().orc_growth_unnorm(om, 1.0) == pytest.approx(cpt, rel=5e-3)


@pytest.mark.parametrize("om", [0.25, 0.3, 0.35, 1.0])
def test_generator_growth_table_vs_oracle(orc, om):
    a, D = growth_table(om)
    idx = np.arange(0, 512, 17)
    for i in idx:
        assert D[i] == pytest.approx(orc.lib().orc_growth_D(om, a[i]), rel=1e-10)
    assert D[-1] == 1.0 and a[0] == 1e-3 and a[-1] == 1.0


def test_growth_inversion(orc):
    a, D = growth_table(1.0)          # EdS: a(D) = D, linear data
    g = orc.Growth(a, D)
    q = np.array([1e-3, 0.01, 0.5, 0.99999, 1.0])
    assert np.allclose(orc.growth_invert(g.D, g.a, g.M, q), q, rtol=1e-12)
    assert orc.growth_invert(g.D, g.a, g.M, [1.5])[0] == np.inf
    assert orc.growth_invert(g.D, g.a, g.M, [1e-5])[0] == 1e-3
    a, D = growth_table(0.3)
    g = orc.Growth(a, D)
    # knots map back to themselves
    got = orc.growth_invert(g.D, g.a, g.M, D[::37])
    assert np.allclose(got, a[::37], rtol=1e-14)


def test_max_over_radii_brute_force(orc):
    cosmo = Cosmology()
    radii = [8.0, 4.0, 2.0, 1.0]
    slabs = [h.numpy() for _, h in hessian_slabs(16, 50.0, radii, 21, cosmo)]
    a, D = growth_table(0.3)
    g = orc.Growth(a, D)
    Fmax, Rmax, acoll = orc.collapse(slabs, g)
    Fs = np.stack([orc.points(h)[1] for h in slabs])          # (R, n)
    best = np.max(Fs, axis=0)
    arg = np.argmax(Fs, axis=0)                               # first maximum wins
    collapsed = best > 0
    assert np.array_equal(Fmax, np.where(collapsed, best, 0.0))
    assert np.array_equal(Rmax, np.where(collapsed, arg, -1).astype(np.int32))
    expect_a = orc.growth_invert(g.D, g.a, g.M, 1.0 / best[collapsed])
    assert np.allclose(acoll[collapsed], expect_a, rtol=1e-12)
    assert np.all(np.isinf(acoll[~collapsed]))
    # earliest collapse: max F is min D_c, so min a_c
    acs = np.stack([np.where(F > 0, orc.growth_invert(g.D, g.a, g.M, np.where(F > 0, 1 / np.where(F > 0, F, 1), 2.0)), np.inf) for F in Fs])
    assert np.allclose(acoll[collapsed], np.min(acs, axis=0)[collapsed], rtol=1e-12)


def test_max_ties_and_nan(orc):
    h = table_grid_hessians(*table_knots(1.0, 4, 4, 4))
    a, D = growth_table(0.3)
    g = orc.Growth(a, D)
    Fmax, Rmax, acoll = orc.collapse([h, h, h], g)            # exact ties
    assert np.all(Rmax[Fmax > 0] == 0)
    bad = h.copy()
    bad[0, :5] = np.nan
    bad[3, 5:9] = np.inf
    F2, R2, a2 = Fmax.copy(), Rmax.copy(), acoll.copy()
    orc.update_radius(bad * 10.0, 7, g, F2, R2, a2, reset=False)
    assert np.array_equal(F2[:9], Fmax[:9]) and np.array_equal(R2[:9], Rmax[:9])
