"""Pins for the oracle's homogeneous-ellipsoid collapse (the source of the
Tabulated table), CPU only.

  * internal-tide coefficients alpha_i against scipy's adaptive quadrature of
    their defining integral, their sum 2 and the sphere's 2/3;
  * Einstein-de Sitter sphere: the linear density at collapse is
    (3/20)(12 pi)^(2/3) = 1.68647 (the Zel'dovich start at a = 1e-7 shifts it
    by ~1e-7);
  * LCDM sphere (Omega_m = 0.3) and EdS: the collapse time of the same top
    hat integrated by scipy as a single mass shell, d2R/dt2 = -(Om/2)/R^2 +
    (1 - Om) R, from the third-order spherical growing mode at a = 1e-3,
    with the growth factor from scipy's quadrature of the growth integral;
  * Einstein-de Sitter scale invariance: F(s l) = s F(l);
  * early times: the axes follow the Zel'dovich solution 1 - l_i D (an error
    in the sign or the trace of the external tide shows here), and a sphere
    follows the third-order series 1 - u - (3/7) u^2 - (23/63) u^3, u = l D;
  * the oracle's step converges: halving it moves F by < 2e-8;
  * the modified-gravity option (perturbations' gravity scaled by
    mu(a) = 1 + mu0 / E(a)^2): mu0 = 0 is the general-relativity result bit
    for bit; the linear growth against scipy's integration of
    D'' + (2 - 1.5 Om(a)) D' = 1.5 Om(a) mu(a) D; a top hat against scipy's
    mass shell with the perturbation's gravity scaled,
    d2R/dt2 = -(Om/2) a^-3 R (1 + mu delta) + (1 - Om) R, 1 + delta = (a/R)^3;
    from the same initial perturbation, stronger gravity (mu0 > 0) collapses
    every ellipsoid earlier.
"""

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

DELTA_C_EDS = 0.15 * (12 * np.pi) ** (2.0 / 3.0)


def _alpha_quad(x, i):
    j, k = (i + 1) % 3, (i + 2) % 3
    f = lambda t: 1.0 / ((x[i] ** 2 + t) ** 1.5 * np.sqrt((x[j] ** 2 + t) * (x[k] ** 2 + t)))
    s = min(x) ** 2
    v = quad(f, 0, s, epsabs=0, epsrel=1e-13, limit=400)[0] + quad(f, s, np.inf, epsabs=0, epsrel=1e-13,
                                                                     limit=400)[0]
    return abs(np.prod(x)) * v


def test_alpha_vs_quadrature_and_identities(orc):
    rng = np.random.default_rng(4)
    for _ in range(60):
        x = np.exp(rng.uniform(-5, 1, 3))
        al = [orc.ell_alpha(x, i) for i in range(3)]
        for i in range(3):
            ref = _alpha_quad(x, i)
            assert abs(al[i] - ref) <= 1e-11 * max(ref, 1e-3)
        assert abs(sum(al) - 2.0) <= 1e-13
    assert abs(orc.ell_alpha([0.7, 0.7, 0.7], 0) - 2.0 / 3.0) <= 1e-14


def test_eds_sphere_delta_c(orc):
    for lam in (1.0, 2.5):
        F, ac = orc.ellipsoid_F([lam] * 3, 1.0)
        assert abs(3 * lam / F - DELTA_C_EDS) <= 3e-7 * lam
    # 3 l D_c fixed: the collapse scale factor in EdS is DELTA_C / (3 l)
    F, ac = orc.ellipsoid_F([1.0] * 3, 1.0)
    assert abs(ac - DELTA_C_EDS / 3.0) <= 1e-6


def _lcdm_sphere_reference(lam, om, a_s=1e-3):
    """Top hat of linear eigenvalue lam (all three) in flat LCDM by scipy: a
    mass shell of unit Lagrangian radius, d2R/dt2 = -(Om/2)/R^2 + (1 - Om) R,
    started at a_s in the growing mode of the third-order spherical series
    R/a = 1 - u - (3/7) u^2 - (23/63) u^3, u = lam D/D1 (its error there is
    ~u^4 ~ 1e-11), until R reaches 1e-7 a (the remaining free-fall time is
    ~1e-11); D from the growth integral D = (5 Om/2) E int_0^a db/(b E)^3."""
    ol = 1 - om
    E = lambda a: np.sqrt(om / a ** 3 + ol)
    J = lambda a: quad(lambda b: 1.0 / (b * E(b)) ** 3, 0, a, epsabs=0, epsrel=1e-13, limit=200)[0]
    growth = lambda a: 2.5 * om * E(a) * J(a)
    D1 = growth(1.0)
    dE = -1.5 * om / a_s ** 4 / E(a_s)
    dDda = 2.5 * om * (dE * J(a_s) + E(a_s) / (a_s * E(a_s)) ** 3)
    u = lam * growth(a_s) / D1
    du = lam * dDda * a_s * E(a_s) / D1      # du/dt
    R0 = a_s * (1 - u - 3.0 / 7.0 * u ** 2 - 23.0 / 63.0 * u ** 3)
    V0 = a_s * E(a_s) * R0 / a_s + a_s * (-1 - 6.0 / 7.0 * u - 23.0 / 21.0 * u ** 2) * du

    def rhs(t, y):
        a, R, V = y
        return [a * E(a), V, -0.5 * om / R ** 2 + ol * R]

    ev = lambda t, y: y[1] - 1e-7 * y[0]
    ev.terminal = True
    sol = solve_ivp(rhs, [0, 50], [a_s, R0, V0], method="DOP853", rtol=1e-13, atol=1e-30, events=ev)
    a_c = sol.y_events[0][0][0]
    return D1 / growth(a_c), a_c


def test_lcdm_sphere_vs_mass_shell(orc):
    for om, lam in ((0.3, 0.8), (0.3, 2.0), (1.0, 0.8)):
        F_ref, a_ref = _lcdm_sphere_reference(lam, om)
        F, ac = orc.ellipsoid_F([lam] * 3, om)
        # the oracle starts in the Zel'dovich mode at a = 1e-7 (its error
        # ~0.6 lam 1e-7 relative)
        assert abs(F / F_ref - 1) <= 3e-7 * lam, (lam, F, F_ref)
        assert abs(ac / a_ref - 1) <= 3e-7 * lam


def test_eds_scale_invariance(orc):
    for lam in ([1.0, 0.5, -0.2], [2.0, 0.1, -1.5], [0.6, 0.6, 0.1]):
        F1, _ = orc.ellipsoid_F(lam, 1.0)
        F2, _ = orc.ellipsoid_F(2.0 * np.asarray(lam), 1.0)
        assert F1 > 0
        assert abs(F2 / (2.0 * F1) - 1) <= 2e-6


def test_early_times_follow_lpt(orc):
    lam = np.array([3.0, 1.0, -2.0])
    for om in (1.0, 0.3):
        x, d = orc.ellipsoid_axes(lam, om, 1e-3)
        for i in range(3):
            assert abs(x[i] - (1 - lam[i] * d)) <= 3 * (lam[i] * d) ** 2 + 1e-12
        # the first-order term is right to far below the second-order size
        assert abs(x[0] - (1 - lam[0] * d)) > 1e-9
    # a sphere follows the third-order spherical series
    for l in (0.5, 1.0):
        x, d = orc.ellipsoid_axes([l] * 3, 1.0, 0.02)
        u = l * d
        series = 1 - u - 3.0 / 7.0 * u ** 2 - 23.0 / 63.0 * u ** 3
        assert abs(x[0] - series) <= 5 * u ** 4


def test_oracle_step_converged(orc):
    for lam, om in (([1.0, 0.5, -0.2], 0.3), ([1.0, 0.999, 0.998], 0.3), ([0.9, 0.2, 0.1], 1.0)):
        F1, _ = orc.ellipsoid_F(lam, om)
        F2, _ = orc.ellipsoid_F(lam, om, step=orc.ELL_STEP / 2, kappa=orc.ELL_KAPPA / 2)
        assert abs(F1 / F2 - 1) <= 2e-8


def test_no_collapse_of_underdense_ellipsoids(orc):
    F, ac = orc.ellipsoid_F([-0.1, -0.3, -0.5], 0.3)
    assert F == 0.0 and ac == orc.ELL_A_STOP


def _mu(om, mu0, a):
    return 1.0 + mu0 / (om / a ** 3 + 1.0 - om)


def _mg_growth(om, mu0):
    """Growing mode of D'' + (2 - 1.5 Om(a)) D' - 1.5 Om(a) mu(a) D = 0 in
    s = ln a (scipy, dense), started in the EdS mode D = a at a = 1e-8
    (mu - 1 ~ 1e-24 there); returns D(a) for scalar a."""
    def rhs(s, y):
        a = np.exp(s)
        oma = om / a ** 3 / (om / a ** 3 + 1.0 - om)
        return [y[1], -(2.0 - 1.5 * oma) * y[1] + 1.5 * oma * _mu(om, mu0, a) * y[0]]
    s0 = np.log(1e-8)
    sol = solve_ivp(rhs, [s0, np.log(12.0)], [1e-8, 1e-8], method="DOP853", rtol=1e-13, atol=1e-30,
                    dense_output=True)
    return lambda a: sol.sol(np.log(a))[0]


def _mg_sphere_reference(lam, om, mu0, a_s=1e-3):
    """Top hat of linear eigenvalue lam in flat LCDM with the perturbation's
    gravity scaled by mu(a): scipy mass shell in cosmic time,
    d2R/dt2 = -(Om/2) a^-3 R (1 + mu delta) + (1 - Om) R, 1 + delta = (a/R)^3,
    started at a_s in the third-order spherical growing mode (mu - 1 ~ 1e-9
    there), until R = 1e-7 a; D from _mg_growth, normalised at a = 1."""
    ol = 1 - om
    E = lambda a: np.sqrt(om / a ** 3 + ol)
    D = _mg_growth(om, mu0)
    D1 = D(1.0)
    eps = 1e-6
    u = lam * D(a_s) / D1
    dlnD = (np.log(D(a_s * (1 + eps))) - np.log(D(a_s * (1 - eps)))) / (2 * eps)
    du = u * dlnD * E(a_s)                   # du/dt = u (dlnD/dlna) H
    R0 = a_s * (1 - u - 3.0 / 7.0 * u ** 2 - 23.0 / 63.0 * u ** 3)
    V0 = a_s * E(a_s) * R0 / a_s + a_s * (-1 - 6.0 / 7.0 * u - 23.0 / 21.0 * u ** 2) * du

    def rhs(t, y):
        a, R, V = y
        delta = (a / R) ** 3 - 1.0
        return [a * E(a), V, -0.5 * om / a ** 3 * R * (1.0 + _mu(om, mu0, a) * delta) + ol * R]

    ev = lambda t, y: y[1] - 1e-7 * y[0]
    ev.terminal = True
    sol = solve_ivp(rhs, [0, 50], [a_s, R0, V0], method="DOP853", rtol=1e-13, atol=1e-30, events=ev)
    a_c = sol.y_events[0][0][0]
    return D1 / D(a_c), a_c


def test_mg_zero_is_general_relativity(orc):
    for lam in ([1.0, 0.5, -0.2], [2.0, 2.0, 2.0], [0.3, -0.1, -0.4]):
        assert orc.ellipsoid_F(lam, 0.3, mu0=0.0) == orc.ellipsoid_F(lam, 0.3)
    assert orc.ellipsoid_growth1(0.3, 0.0) == orc.ellipsoid_growth1(0.3)


@pytest.mark.parametrize("mu0", [0.5, -0.3])
def test_mg_linear_growth_vs_scipy(orc, mu0):
    # the oracle's D(1) of the mode started as D = a at 1e-7, against scipy's
    ref = _mg_growth(0.3, mu0)(1.0)
    got = orc.ellipsoid_growth1(0.3, mu0)
    assert abs(got / ref - 1) <= 1e-8, (got, ref)
    # gravity stronger today: more growth (and weaker: less)
    assert (got > orc.ellipsoid_growth1(0.3)) == (mu0 > 0)


@pytest.mark.parametrize("mu0", [0.5, -0.3])
def test_mg_sphere_vs_mass_shell(orc, mu0):
    for lam in (0.8, 2.0):
        F_ref, a_ref = _mg_sphere_reference(lam, 0.3, mu0)
        F, ac = orc.ellipsoid_F([lam] * 3, 0.3, mu0=mu0)
        assert abs(F / F_ref - 1) <= 3e-7 * lam, (lam, F, F_ref)
        assert abs(ac / a_ref - 1) <= 3e-7 * lam


def test_mg_stronger_gravity_collapses_earlier(orc):
    # the same initial perturbation (the eigenvalues are linear amplitudes
    # today, so they scale with the option's own D(1)): stronger gravity of
    # the perturbations collapses every ellipsoid earlier
    d0 = orc.ellipsoid_growth1(0.3)
    for lam in ([1.0, 0.5, -0.2], [0.8, 0.8, 0.8], [2.0, -0.5, -1.0]):
        acs = [orc.ellipsoid_F(np.asarray(lam) * orc.ellipsoid_growth1(0.3, m) / d0, 0.3, mu0=m)[1]
               for m in (-0.3, 0.0, 0.5)]
        assert acs[0] > acs[1] > acs[2], (lam, acs)


def test_synth_mg_growth_table_vs_scipy():
    """The growth table the generator writes for the modified-gravity option
    (the table that inverts D_c) against scipy's integration of the same
    equation."""
    import synth
    for mu0 in (0.4, -0.3):
        a, D = synth.growth_table(0.3, mu0=mu0)
        ref = _mg_growth(0.3, mu0)
        Dr = np.array([ref(x) for x in a]) / ref(1.0)
        assert np.max(np.abs(D / Dr - 1)) <= 1e-9
