"""Coefficients of the polynomial used by cos_acos3 (device_collapse.h).

c(r) = cos(acos(r)/3) on r in [-1, 1] is, as a function of
t = sqrt((1 + r)/2) = cos(acos(r)/2), the analytic function cos(2 acos(t)/3)
on t in [0, 1] (its only singularity is at t = -1), so a low-degree
polynomial in t approximates it uniformly, also next to r = -1 where c(r)
itself has a square-root branch point.  The fit is least squares in the
relative error on Chebyshev nodes, refined by Lawson reweighting towards
minimax.  Run: python gen_cos_acos3.py [degree]
"""

import sys

import numpy as np


def fit(degree=7, nodes=4000, lawson=40):
    t = 0.5 + 0.5 * np.cos(np.pi * (np.arange(nodes) + 0.5) / nodes)
    f = np.cos(2.0 * np.arccos(t) / 3.0)
    V = np.vander(t, degree + 1, increasing=True) / f[:, None]
    w = np.ones(nodes)
    for _ in range(lawson):
        c, *_ = np.linalg.lstsq(V * np.sqrt(w)[:, None], np.sqrt(w), rcond=None)
        e = np.abs(V @ c - 1.0)
        w = w * e
        w /= w.sum()
    tt = np.linspace(0.0, 1.0, 400001)
    ff = np.cos(2.0 * np.arccos(tt) / 3.0)
    err = np.max(np.abs(np.polyval(c[::-1], tt) - ff) / ff)
    return c, err


if __name__ == "__main__":
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 7
    c, err = fit(deg)
    print(f"// degree {deg}, max relative error {err:.2e} on [0, 1]")
    for k, v in enumerate(c):
        print(f"    c{k} = {v:.17g}")
