"""Oracle for the collapse-time path (TEST INFRASTRUCTURE ONLY).

A plain FP64 CPU implementation of what the path computes, in C
(collapse_oracle.c) behind ctypes, plus a numpy FP64 multilayer perceptron for
the surrogate's gradient checks (mlp.py).  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the HIP library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "collapse_oracle.c")
_LIB = os.path.join(_HERE, "liborc_collapse.so")

CLASSIC = 0
TABULATED = 1
CLASSIC_LCDM = 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_eig3.argtypes = [_D, _D]
        L.orc_lpt_axis.argtypes = [_D, ctypes.c_int, _D, _D]
        L.orc_collapse_D.argtypes = [_D, ctypes.POINTER(ctypes.c_int)]
        L.orc_collapse_D.restype = ctypes.c_double
        L.orc_classic_F.argtypes = [_D]
        L.orc_classic_F.restype = ctypes.c_double
        L.orc_spline_natural.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_spline_natural.restype = ctypes.c_int
        L.orc_spline_eval.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double]
        L.orc_spline_eval.restype = ctypes.c_double
        L.orc_growth_invert.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double]
        L.orc_growth_invert.restype = ctypes.c_double
        L.orc_table_F.argtypes = [ctypes.c_int] * 3 + [_D] * 5 + [_D]
        L.orc_table_F.restype = ctypes.c_double
        L.orc_table_build.argtypes = [ctypes.c_int] * 3 + [_D] * 3
        L.orc_table_build.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_update_radius.argtypes = ([ctypes.c_int64] + [_D] * 6 + [ctypes.c_int32, ctypes.c_int, ctypes.c_int]
                                        + [_D] * 3 + [ctypes.c_int] * 3 + [_D] * 5
                                        + [ctypes.c_int, _D, _I32, _D])
        L.orc_points.argtypes = [ctypes.c_int64, _D, _D, _D]
        L.orc_growth_unnorm.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_growth_unnorm.restype = ctypes.c_double
        L.orc_growth_D.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_growth_D.restype = ctypes.c_double
        L.orc_lpt_growth.argtypes = [ctypes.c_double, ctypes.c_int, _D, _D, _D, _D]
        L.orc_lpt_growth.restype = ctypes.c_int
        L.orc_collapse_D_lcdm.argtypes = [_D, ctypes.c_int] + [_D] * 7 + [ctypes.POINTER(ctypes.c_int)]
        L.orc_collapse_D_lcdm.restype = ctypes.c_double
        L.orc_update_radius_lcdm.argtypes = ([ctypes.c_int64] + [_D] * 6 + [ctypes.c_int32, ctypes.c_int]
                                             + [_D] * 9 + [ctypes.c_int, _D, _I32, _D])
        L.orc_g_lcdm.argtypes = [_D, ctypes.c_int] + [_D] * 7 + [ctypes.c_double, _D]
        L.orc_g_lcdm.restype = ctypes.c_double
        L.orc_ell_alpha.argtypes = [_D, ctypes.c_int]
        L.orc_ell_alpha.restype = ctypes.c_double
        L.orc_ellipsoid_F.argtypes = [_D] + [ctypes.c_double] * 6 + [_D]
        L.orc_ellipsoid_F.restype = ctypes.c_double
        L.orc_ellipsoid_axes.argtypes = [_D] + [ctypes.c_double] * 5 + [_D, _D]
        L.orc_ellipsoid_table.argtypes = [ctypes.c_int] * 3 + [_D] * 3 + [ctypes.c_double] * 6 + [_D]
        L.orc_ell_growth1.argtypes = [ctypes.c_double] * 4
        L.orc_ell_growth1.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """Threads for the parallel loops that follow (timing only)."""
    lib().orc_set_threads(int(n))


def eig3(h):
    """Sorted (descending) eigenvalues of one Hessian h = (xx,yy,zz,xy,xz,yz)."""
    h = _f64(h)
    lam = np.empty(3)
    lib().orc_eig3(_p(h), _p(lam))
    return lam


def lpt_axis(lam, axis=0):
    """(b_i, c_i): second- and third-order LPT coefficients of axis i."""
    lam = _f64(lam)
    b, c = ctypes.c_double(), ctypes.c_double()
    lib().orc_lpt_axis(_p(lam), int(axis), ctypes.byref(b), ctypes.byref(c))
    return b.value, c.value


def collapse_D(lam):
    """Growth factor at collapse for sorted eigenvalues, or None."""
    lam = _f64(lam)
    found = ctypes.c_int()
    D = lib().orc_collapse_D(_p(lam), ctypes.byref(found))
    return D if found.value else None


def classic_F(lam):
    lam = _f64(lam)
    return lib().orc_classic_F(_p(lam))


def spline_natural(x, y):
    x, y = _f64(x), _f64(y)
    M = np.empty_like(x)
    if lib().orc_spline_natural(len(x), _p(x), _p(y), _p(M)) != 0:
        raise ValueError("knots must be strictly increasing and at least 2")
    return M


def spline_eval(x, y, M, q):
    x, y, M = _f64(x), _f64(y), _f64(M)
    L = lib()
    return np.array([L.orc_spline_eval(len(x), _p(x), _p(y), _p(M), float(v)) for v in np.atleast_1d(q)])


def growth_invert(D, a, M, Dc):
    D, a, M = _f64(D), _f64(a), _f64(M)
    L = lib()
    return np.array([L.orc_growth_invert(len(D), _p(D), _p(a), _p(M), float(v)) for v in np.atleast_1d(Dc)])


def table_build(dk, F):
    """F shaped (nx, ny, nd) -> second derivatives of each delta row."""
    F = _f64(F)
    dk = _f64(dk)
    nx, ny, nd = F.shape
    M = np.empty_like(F)
    if lib().orc_table_build(nx, ny, nd, _p(dk), _p(F), _p(M)) != 0:
        raise ValueError("bad table knots")
    return M


def table_F(xk, yk, dk, F, M, lam):
    xk, yk, dk, F, M, lam = map(_f64, (xk, yk, dk, F, M, lam))
    nx, ny, nd = F.shape
    return lib().orc_table_F(nx, ny, nd, _p(xk), _p(yk), _p(dk), _p(F), _p(M), _p(lam))


def points(h6):
    """Per point: sorted eigenvalues (n, 3) and Classic F (n,).  h6 is (6, n)."""
    h6 = _f64(h6)
    n = h6.shape[1]
    lam = np.empty((n, 3))
    F = np.empty(n)
    lib().orc_points(n, _p(h6), _p(lam), _p(F))
    return lam, F


def lpt_growth(omega_m, a):
    """Ratios (k2, k3a, k3b) of the second- and third-order LPT growth of flat
    LCDM to their Einstein-de Sitter values at the scale factors a."""
    a = _f64(a)
    k = [np.empty_like(a) for _ in range(3)]
    if lib().orc_lpt_growth(float(omega_m), len(a), _p(a), *[_p(x) for x in k]) != 0:
        raise ValueError("need omega_m > 0 and a strictly increasing, > 0")
    return tuple(k)


class Growth:
    """Inverse growth spline a(D) built from a growth table (a_k, D_k).  With
    omega_m, also the LCDM time coefficients of the LPT collapse at the knots
    and their natural splines in D (the Classic method with LCDM
    coefficients)."""

    def __init__(self, a, D, omega_m=None):
        self.a = _f64(a)
        self.D = _f64(D)
        self.M = spline_natural(self.D, self.a)
        self.omega_m = omega_m
        if omega_m is not None:
            self.k2, self.k3a, self.k3b = lpt_growth(omega_m, self.a)
            self.m2, self.m3a, self.m3b = (spline_natural(self.D, k) for k in (self.k2, self.k3a, self.k3b))

    def _kappa_args(self):
        if self.omega_m is None:
            raise ValueError("this growth table has no LCDM coefficients (pass omega_m)")
        return [_p(x) for x in (self.D, self.k2, self.m2, self.k3a, self.m3a, self.k3b, self.m3b)]


# the homogeneous-ellipsoid integration: start, stop and the oracle's step
# (in ln a) and step limit near collapse
ELL_A_I = 1e-7
ELL_A_STOP = 10.0
ELL_STEP = 2e-3
ELL_KAPPA = 0.02


def ell_alpha(x, i):
    """Internal-tide coefficient alpha_i of an ellipsoid with axes x."""
    return lib().orc_ell_alpha(_p(_f64(x)), int(i))


def ellipsoid_F(lam, omega_m, step=ELL_STEP, kappa=ELL_KAPPA, a_i=ELL_A_I, a_stop=ELL_A_STOP, mu0=0.0):
    """(F = 1/D_c, a_c) of the homogeneous ellipsoid with eigenvalues lam;
    mu0: the modified-gravity option, perturbations' gravity scaled by
    mu(a) = 1 + mu0 / E(a)^2 (0: general relativity)."""
    ac = ctypes.c_double()
    F = lib().orc_ellipsoid_F(_p(_f64(lam)), float(omega_m), float(mu0), float(a_i), float(a_stop), float(step),
                              float(kappa), ctypes.byref(ac))
    return F, ac.value


def ellipsoid_axes(lam, omega_m, a_out, step=ELL_STEP, a_i=ELL_A_I, mu0=0.0):
    """(axes x_i = R_i/a, D/D1) of the ellipsoid at a_out."""
    x = np.empty(3)
    d = ctypes.c_double()
    lib().orc_ellipsoid_axes(_p(_f64(lam)), float(omega_m), float(mu0), float(a_i), float(a_out), float(step),
                             _p(x), ctypes.byref(d))
    return x, d.value


def ellipsoid_growth1(omega_m, mu0=0.0, step=ELL_STEP, a_i=ELL_A_I):
    """D(a = 1) of the growing mode started as D = a at a_i (the
    normalisation of the ellipsoid's linear growth), with the same mu."""
    return lib().orc_ell_growth1(float(omega_m), float(mu0), float(a_i), float(step))


def ellipsoid_table(xk, yk, dk, omega_m, step=ELL_STEP, kappa=ELL_KAPPA, a_i=ELL_A_I, a_stop=ELL_A_STOP,
                    mu0=0.0):
    """F over the nodes of knots (already scaled), shaped (nx, ny, nd)."""
    xk, yk, dk = _f64(xk), _f64(yk), _f64(dk)
    F = np.empty((len(xk), len(yk), len(dk)))
    lib().orc_ellipsoid_table(len(xk), len(yk), len(dk), _p(xk), _p(yk), _p(dk), float(omega_m), float(mu0),
                              float(a_i), float(a_stop), float(step), float(kappa), _p(F))
    return F


def collapse_D_lcdm(lam, growth: Growth):
    """Growth factor at collapse with the LCDM time coefficients, or None."""
    lam = _f64(lam)
    found = ctypes.c_int()
    D = lib().orc_collapse_D_lcdm(_p(lam), len(growth.D), *growth._kappa_args(), ctypes.byref(found))
    return D if found.value else None


def g_lcdm(lam, growth: Growth, D):
    """(G(D), dG/dD) of the LCDM collapse condition."""
    lam = _f64(lam)
    d = ctypes.c_double()
    g = lib().orc_g_lcdm(_p(lam), len(growth.D), *growth._kappa_args(), float(D), ctypes.byref(d))
    return g, d.value


class Table:
    """Tabulated F over knots (x, y, delta); F shaped (nx, ny, nd)."""

    def __init__(self, xk, yk, dk, F):
        self.xk, self.yk, self.dk = _f64(xk), _f64(yk), _f64(dk)
        self.F = _f64(F)
        self.M = table_build(self.dk, self.F)


def update_radius(h6, radius_index, growth: Growth, Fmax, Rmax, acoll, reset, method=CLASSIC,
                  table: Table | None = None):
    """Apply one smoothing radius to the running maxima (in place).
    h6: (6, n) float64; Fmax float64[n], Rmax int32[n], acoll float64[n] or None."""
    h6 = _f64(h6)
    n = h6.shape[1]
    assert Fmax.dtype == np.float64 and Fmax.flags.c_contiguous and Fmax.shape == (n,)
    assert Rmax.dtype == np.int32 and Rmax.flags.c_contiguous and Rmax.shape == (n,)
    if acoll is not None:
        assert acoll.dtype == np.float64 and acoll.flags.c_contiguous and acoll.shape == (n,)
    null = ctypes.cast(None, _D)
    if method == CLASSIC_LCDM:
        lib().orc_update_radius_lcdm(n, *[_p(h6[c]) for c in range(6)], int(radius_index), len(growth.D),
                                     _p(growth.D), _p(growth.a), _p(growth.M),
                                     *growth._kappa_args()[1:], int(bool(reset)), _p(Fmax),
                                     Rmax.ctypes.data_as(_I32), _p(acoll) if acoll is not None else null)
        return
    if method == TABULATED:
        t = table
        nx, ny, nd = t.F.shape
        targs = (nx, ny, nd, _p(t.xk), _p(t.yk), _p(t.dk), _p(t.F), _p(t.M))
    else:
        targs = (0, 0, 0, null, null, null, null, null)
    lib().orc_update_radius(n, *[_p(h6[c]) for c in range(6)], int(radius_index), int(method),
                            len(growth.D), _p(growth.D), _p(growth.a), _p(growth.M), *targs,
                            int(bool(reset)), _p(Fmax), Rmax.ctypes.data_as(_I32),
                            _p(acoll) if acoll is not None else null)


def collapse(slabs, growth: Growth, method=CLASSIC, tables=None, with_acoll=True):
    """Run every radius in order.  slabs: iterable of (6, n) arrays.
    Returns (Fmax, Rmax, acoll)."""
    Fmax = Rmax = acoll = None
    for r, h6 in enumerate(slabs):
        h6 = _f64(h6)
        if Fmax is None:
            n = h6.shape[1]
            Fmax = np.zeros(n)
            Rmax = np.full(n, -1, dtype=np.int32)
            acoll = np.full(n, np.inf) if with_acoll else None
        update_radius(h6, r, growth, Fmax, Rmax, acoll, reset=(r == 0), method=method,
                      table=None if tables is None else tables[r])
    return Fmax, Rmax, acoll
