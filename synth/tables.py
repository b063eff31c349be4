"""Knot grids of the tabulated collapse function and the points they sample.

Sec. 3 of the paper: collapse times are tabulated on a grid of eigenvalues in
the coordinates delta = l1 + l2 + l3, x = l1 - l2, y = l2 - l3 (eigenvalues in
descending order), with non-uniform sampling along delta; the toy code of
Sec. 4.3 uses a 64 x 64 grid in (x, y) whose nodes each carry a 128-knot spline
in delta.

Readings (ranges are not given): knots scale with sigma(R) of the smoothing
radius; x, y uniform in [0, 6 sigma]; delta in [-6 sigma, 8 sigma] with a sinh
stretch that puts the knots closest together near delta = sigma.

`table_grid_hessians` returns diagonal Hessians whose eigenvalues are the
table's sample points, so that any collapse solver fed with Hessians can fill
the table: for a node (delta, x, y) the diagonal is
((delta + 2x + y)/3, (delta - x + y)/3, (delta - x - 2y)/3).
"""

from __future__ import annotations

import numpy as np


def table_knots(sigma: float = 1.0, nx: int = 64, ny: int = 64, nd: int = 128):
    """Return (x[nx], y[ny], delta[nd]) float64 knot arrays, strictly increasing."""
    x = np.linspace(0.0, 6.0 * sigma, nx)
    y = np.linspace(0.0, 6.0 * sigma, ny)
    t = np.linspace(0.0, 1.0, nd)
    d = sigma * (1.0 + 7.0 * np.sinh(3.0 * (t - 0.5)) / np.sinh(1.5))
    return x, y, d


def table_grid_hessians(x, y, d):
    """(6, nx*ny*nd) SoA of diagonal Hessians, node order [ix][iy][id]."""
    X, Y, Dl = np.meshgrid(np.asarray(x, np.float64), np.asarray(y, np.float64),
                           np.asarray(d, np.float64), indexing="ij")
    h = np.zeros((6, X.size), dtype=np.float64)
    h[0] = ((Dl + 2.0 * X + Y) / 3.0).ravel()
    h[1] = ((Dl - X + Y) / 3.0).ravel()
    h[2] = ((Dl - X - 2.0 * Y) / 3.0).ravel()
    return h
