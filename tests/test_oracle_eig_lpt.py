"""Pins for the oracle's eigenvalues and its Classic collapse (CPU only).

Eigenvalues (Sec. 3, sorted descending) are pinned by the matrix invariants,
by numpy's symmetric eigensolver and by exact special cases.

The collapse condition is the LPT reading written up in the design notes; it
is pinned by facts that do not depend on how the oracle codes it:
  * second-order trace condition of LPT: sum_i b_i = -(3/7) mu_2;
  * third-order trace condition: sum_i c_i = -(5/9) sum_{i!=j} a_i b_j
    + (1/3) l1 l2 l3, i.e. the -1/3 det and -10/21 mixed-invariant sources;
  * the sphere: (R/q)^-3 must reproduce the exact spherical-collapse series
    1 + delta + (17/21) delta^2 + (341/567) delta^3;
  * plane-parallel (l2 = l3 = 0): the Zel'dovich solution is exact, D_c = 1/l1;
  * homogeneity D_c(s l) = D_c(l) / s;
  * l1 <= 0 never collapses;
  * brute force: a dense sign scan plus 60-digit bisection of the axis-1 cubic
    written in its collapsed form (beta, gamma in l1, s = l2 + l3, p = l2 l3),
    an expression the oracle never uses.
"""

import mpmath
import numpy as np
import pytest


def _sym(h):
    xx, yy, zz, xy, xz, yz = h
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def _random_hessians(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 6)) * scale


def test_eig_invariants_and_numpy(orc):
    for h in _random_hessians(2000, 11, 1.7):
        lam = orc.eig3(h)
        H = _sym(h)
        norm = np.linalg.norm(H)
        assert lam[0] >= lam[1] >= lam[2]
        assert abs(lam.sum() - np.trace(H)) <= 1e-13 * norm
        assert abs((lam ** 2).sum() - (H * H).sum()) <= 1e-13 * norm ** 2
        assert abs(lam.prod() - np.linalg.det(H)) <= 1e-12 * norm ** 3
        ref = np.linalg.eigvalsh(H)[::-1]
        assert np.max(np.abs(lam - ref)) <= 1e-13 * norm


def test_eig_special_cases(orc):
    assert list(orc.eig3([3.0, -1.0, 2.0, 0, 0, 0])) == [3.0, 2.0, -1.0]
    assert list(orc.eig3([0.7, 0.7, 0.7, 0, 0, 0])) == [0.7, 0.7, 0.7]
    assert list(orc.eig3([0.0] * 6)) == [0.0, 0.0, 0.0]
    # rank-one (planar) matrix v v^T: eigenvalues (|v|^2, 0, 0)
    v = np.array([1.0, 2.0, -2.0])
    H = np.outer(v, v)
    lam = orc.eig3([H[0, 0], H[1, 1], H[2, 2], H[0, 1], H[0, 2], H[1, 2]])
    assert abs(lam[0] - 9.0) < 1e-14 and abs(lam[1]) < 1e-14 and abs(lam[2]) < 1e-14
    # repeated eigenvalue with a rotated frame
    Q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
    H = Q @ np.diag([2.0, 2.0, -1.0]) @ Q.T
    lam = orc.eig3([H[0, 0], H[1, 1], H[2, 2], H[0, 1], H[0, 2], H[1, 2]])
    assert np.allclose(lam, [2.0, 2.0, -1.0], atol=1e-14)


def test_lpt_trace_conditions(orc):
    rng = np.random.default_rng(5)
    for _ in range(500):
        lam = np.sort(rng.normal(size=3))[::-1]
        bc = [orc.lpt_axis(lam, i) for i in range(3)]
        b = np.array([x[0] for x in bc])
        c = np.array([x[1] for x in bc])
        a = -lam
        mu2 = lam[0] * lam[1] + lam[0] * lam[2] + lam[1] * lam[2]
        assert abs(b.sum() + 3.0 / 7.0 * mu2) < 1e-14
        mixed = sum(a[i] * b[j] for i in range(3) for j in range(3) if i != j)
        assert abs(c.sum() - (-5.0 / 9.0 * mixed + lam.prod() / 3.0)) < 1e-14


def test_lpt_sphere_reproduces_spherical_series(orc):
    # R/q = 1 + (-lam) D + b D^2 + c D^3 with delta_lin = 3 lam D; the
    # density 1 + delta_NL = (R/q)^-3 must match the exact spherical series
    lam = 0.37
    b, c = orc.lpt_axis([lam, lam, lam], 0)
    # in units of delta_lin: R/q = 1 - d/3 + (b/(9 lam^2)) d^2 + (c/(27 lam^3)) d^3
    e1, e2, e3 = -1.0 / 3.0, b / (9 * lam ** 2), c / (27 * lam ** 3)
    # series of (1 + x)^-3 with x = e1 d + e2 d^2 + e3 d^3, to third order
    s1 = -3 * e1
    s2 = -3 * e2 + 6 * e1 ** 2
    s3 = -3 * e3 + 12 * e1 * e2 - 10 * e1 ** 3
    assert abs(s1 - 1.0) < 1e-15
    assert abs(s2 - 17.0 / 21.0) < 1e-14
    assert abs(s3 - 341.0 / 567.0) < 1e-14


def test_sphere_closed_form_root(orc):
    # sphere: R/q = 1 - u - (3/7) u^2 - (23/63) u^3, u = lam D; the collapse
    # is its real root (Cardano, the cubic has one real root here)
    a3, a2, a1, a0 = mpmath.mpf(-23) / 63, mpmath.mpf(-3) / 7, mpmath.mpf(-1), mpmath.mpf(1)
    mpmath.mp.dps = 40
    roots = mpmath.polyroots([a3, a2, a1, a0], maxsteps=200, extraprec=200)
    real = [r.real for r in roots if abs(r.imag) < mpmath.mpf(10) ** -30 and r.real > 0]
    u_c = float(min(real))
    for lam in (0.01, 0.5, 1.0, 3.7, 250.0):
        D = orc.collapse_D([lam, lam, lam])
        assert D is not None
        assert abs(D * lam - u_c) <= 4e-16 * u_c
    # linear density contrast at collapse of this third-order reading,
    # between the Zel'dovich value 3 and the exact spherical 1.686
    assert abs(3 * u_c - 2.05008378247626) < 1e-13


def test_planar_is_zeldovich(orc):
    for l1 in (1e-3, 0.2, 1.0, 7.5, 1e3):
        D = orc.collapse_D([l1, 0.0, 0.0])
        assert D == pytest.approx(1.0 / l1, rel=2e-16)


def test_homogeneity(orc):
    rng = np.random.default_rng(7)
    for _ in range(300):
        lam = np.sort(rng.normal(size=3))[::-1]
        if lam[0] <= 0:
            continue
        D = orc.collapse_D(lam)
        for s in (0.25, 2.0, 1024.0):   # powers of two: exact scaling in binary
            Ds = orc.collapse_D(lam * s)
            assert Ds == pytest.approx(D / s, rel=1e-15)


def test_nonpositive_l1_never_collapses(orc):
    rng = np.random.default_rng(9)
    for _ in range(5000):
        lam = -np.abs(np.sort(rng.normal(size=3) * rng.uniform(0.01, 10)))[::-1]
        lam = np.sort(lam)[::-1]
        assert orc.collapse_D(lam) is None
    assert orc.collapse_D([0.0, -1.0, -2.0]) is None
    assert orc.collapse_D([0.0, 0.0, 0.0]) is None


def _brute_root(lam, digits=60):
    """Smallest positive root of the axis-1 cubic written in collapsed form,
    by a dense sign scan and high-precision bisection."""
    mpmath.mp.dps = digits
    l1, l2, l3 = (mpmath.mpf(float(v)) for v in lam)   # exact binary values
    s, p = l2 + l3, l2 * l3
    beta = -mpmath.mpf(3) / 14 * l1 * s
    gamma = -l1 * ((l1 * s + 2 * p) / 56 + 17 * s * s / 168 - p / 9)
    g = lambda D: 1 - l1 * D + beta * D ** 2 + gamma * D ** 3
    hi_end = mpmath.mpf(64) / abs(l1) if l1 != 0 else mpmath.mpf(1e6)
    grid = [hi_end * k / 40000 for k in range(1, 40001)]
    prev = mpmath.mpf(0)
    for D in grid:
        if g(D) <= 0:
            lo, hi = prev, D
            for _ in range(250):
                mid = (lo + hi) / 2
                if g(mid) > 0:
                    lo = mid
                else:
                    hi = mid
            return float(hi)
        prev = D
    return None


@pytest.mark.parametrize("lam", [(1, 0.5, 0.25), (2, -0.5, -1), (1, 1, 0), (0.5, 0.2, -0.3),
                                 (3, 2.5, 2.4), (0.3, -2.0, -2.5), (4.0, -0.1, -6.0)])
def test_brute_force_root(orc, lam):
    D = orc.collapse_D(lam)
    ref = _brute_root(lam)
    assert ref is not None and D is not None
    assert abs(D - ref) <= 4e-16 * ref


def test_brute_force_random(orc):
    rng = np.random.default_rng(13)
    for _ in range(6):
        lam = np.sort(rng.normal(size=3))[::-1]
        lam[0] = abs(lam[0]) + 0.05
        lam = np.sort(lam)[::-1]
        D = orc.collapse_D(lam)
        ref = _brute_root(lam, digits=40)
        assert (D is None) == (ref is None)
        if ref is not None:
            assert abs(D - ref) <= 4e-16 * ref
