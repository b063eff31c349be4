"""GPU parity of the FP64 Tabulated path (device rebuild of the delta splines
for every radius, cubic spline in delta + bilinear in (x, y)) against the
oracle.  Tables are filled by the oracle's Classic solve at the table's
sample points; both sides then interpolate the same table."""

import numpy as np
import pytest
import torch

import synth
from tests._helpers import compare, near_tie_mask

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2510_02873_amd as P
    return P


def _filled_table(orc, knots, sigma):
    xk, yk, dk = (np.asarray(k) * sigma for k in knots)
    _, F = orc.points(synth.table_grid_hessians(xk, yk, dk))
    return orc.Table(xk, yk, dk, F.reshape(len(xk), len(yk), len(dk)))


def _run(pkg, orc, knots, slabs, sigmas, a, D, tables=None):
    tabs = tables or [_filled_table(orc, knots, s) for s in sigmas]
    ref = orc.collapse([np.asarray(s) for s in slabs], orc.Growth(a, D), method=orc.TABULATED, tables=tabs)
    per_r = []
    for h, t in zip(slabs, tabs):
        n = h.shape[1]
        F, R, A = np.zeros(n), np.full(n, -1, np.int32), np.full(n, np.inf)
        orc.update_radius(np.asarray(h), 0, orc.Growth(a, D), F, R, A, reset=True, method=orc.TABULATED, table=t)
        per_r.append(F)
    with pkg.Collapse([(a, D)], method=pkg.PINO_TABULATED, table_knots=knots) as col:
        n = slabs[0].shape[1]
        Fm, Rm, ac = col.outputs(n)
        for r, (h, t, s) in enumerate(zip(slabs, tabs, sigmas)):
            tF = torch.from_numpy(np.ascontiguousarray(t.F)).cuda()
            col.apply(torch.as_tensor(np.asarray(h)).cuda(), r, Fm, Rm, ac, reset=(r == 0), sigma_R=s, table_F=tF)
        torch.cuda.synchronize()
        got = (Fm.cpu().numpy(), Rm.cpu().numpy(), ac.cpu().numpy())
    return ref, got, near_tie_mask(per_r)


def test_c1_tabulated(pkg, orc):
    cfg = synth.config("C1")
    slabs = [h.numpy() for _, h in synth.hessian_slabs(cfg["n_side"], cfg["box"], cfg["radii"], cfg["seed"])]
    sigmas = [synth.grid_sigma_gauss(cfg["n_side"], cfg["box"], R) for R in cfg["radii"]]
    a, D = synth.growth_table(0.3)
    knots = synth.table_knots(1.0, 64, 64, 128)
    print(f"C1 tabulated: n={slabs[0].shape[1]} radii={len(slabs)} table 64x64x128", flush=True)
    ref, got, ties = _run(pkg, orc, knots, slabs, sigmas, a, D)
    st = compare(ref, got, tie_mask=ties, label="C1 tabulated")
    print("C1 tabulated stats", st, flush=True)


def test_tabulated_exact_on_bilinear_linear_data(pkg, orc):
    """F = (c0 + c1 x + c2 y + c3 x y)(d0 + d1 delta) is reproduced exactly by
    both sides (the spline is exact on linear data, bilinear on bilinear)."""
    rng = np.random.default_rng(3)
    xk = np.sort(np.concatenate([[0.0, 6.0], rng.uniform(0, 6, 14)]))
    yk = np.sort(np.concatenate([[0.0, 6.0], rng.uniform(0, 6, 10)]))
    dk = np.sort(np.concatenate([[-6.0, 8.0], rng.uniform(-6, 8, 30)]))
    X, Y, Dl = np.meshgrid(xk, yk, dk, indexing="ij")
    fn = lambda x, y, d: (0.3 + 0.2 * x + 0.1 * y + 0.05 * x * y) * (2.0 + 0.1 * d)
    tab = orc.Table(xk, yk, dk, fn(X, Y, Dl))
    n = 20000
    lam = np.sort(rng.normal(size=(n, 3)) * 1.5, axis=1)[:, ::-1]
    h6 = np.zeros((6, n))
    h6[0], h6[1], h6[2] = lam[:, 0], lam[:, 1], lam[:, 2]
    a, D = synth.growth_table(0.3)
    ref, got, _ = _run(pkg, orc, (xk, yk, dk), [h6], [1.0], a, D, tables=[tab])
    compare(ref, got, label="bilinear-linear")
    d, x, y = lam.sum(1), lam[:, 0] - lam[:, 1], lam[:, 1] - lam[:, 2]
    inside = (x <= 6) & (y <= 6) & (d >= -6) & (d <= 8)
    exact = np.maximum(fn(x, y, d), 0.0)
    assert np.allclose(got[0][inside], exact[inside], rtol=1e-12, atol=1e-13)


def test_tabulated_ragged_and_degenerate(pkg, orc):
    rng = np.random.default_rng(9)
    knots = synth.table_knots(1.0, 16, 12, 40)
    a, D = synth.growth_table(0.3)
    for n in (1, 255, 4099):
        h6 = rng.normal(size=(6, n)) * 0.8
        h6[:, 0] = [1.0, 1.0, 1.0, 0, 0, 0]     # spherical: x = y = 0
        ref, got, _ = _run(pkg, orc, knots, [h6], [0.9], a, D)
        compare(ref, got, label=f"tab n={n}")


def test_table_reproduces_classic(pkg, orc):
    """Reported, not gated: interpolating the Classic-filled table recovers
    the Classic D_c to the table's interpolation error."""
    cfg = synth.config("C1")
    h = synth.hessian_radius(cfg["n_side"], cfg["box"], 2.0, cfg["seed"]).numpy()
    sigma = synth.grid_sigma_gauss(cfg["n_side"], cfg["box"], 2.0)
    knots = synth.table_knots(1.0, 64, 64, 128)
    a, D = synth.growth_table(0.3)
    ref, got, _ = _run(pkg, orc, knots, [h], [sigma], a, D)
    _, Fc = orc.points(h)
    m = (Fc > 0.05) & (got[0] > 0)
    rel = np.abs(got[0][m] - Fc[m]) / Fc[m]
    print(f"table vs classic: median rel {np.median(rel):.2e} p99 {np.percentile(rel, 99):.2e}", flush=True)
    assert np.median(rel) < 1e-2


@pytest.mark.parametrize("n", [1, 3, 1001])
def test_tabulated_unaligned_arrays_match_aligned(pkg, orc, n):
    """Arrays that are 8- but not 16-byte aligned take the one-particle-per-
    lane kernel; it equals the paired kernel bit for bit (odd sizes exercise
    the paired kernel's last element)."""
    rng = np.random.default_rng(n + 5)
    knots = synth.table_knots(1.0, 16, 12, 40)
    a, D = synth.growth_table(0.3)
    t = _filled_table(orc, knots, 0.8)
    tF = torch.from_numpy(np.ascontiguousarray(t.F)).cuda()
    slabs = [torch.from_numpy(rng.normal(size=(6, n)) * 0.8).cuda() for _ in range(2)]
    with pkg.Collapse([(a, D)], method=pkg.PINO_TABULATED, table_knots=knots) as col:
        F1, R1, A1 = col.outputs(n)
        bufF = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        bufR = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        bufA = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        F2, R2, A2 = bufF[1:], bufR[1:], bufA[1:]
        for r, hd in enumerate(slabs):
            buf = torch.empty((6, n + 1), dtype=torch.float64, device="cuda")
            buf[:, 1:] = hd
            hu = [buf[c, 1:] for c in range(6)]
            col.apply(hd, r, F1, R1, A1 if r == 1 else None, reset=(r == 0), finalize=(r == 1), sigma_R=0.8,
                      table_F=tF)
            col.apply(hu, r, F2, R2, A2 if r == 1 else None, reset=(r == 0), finalize=(r == 1), sigma_R=0.8,
                      table_F=tF)
        torch.cuda.synchronize()
        assert torch.equal(F1, F2) and torch.equal(R1, R2) and torch.equal(A1, A2)


@pytest.mark.parametrize("spacing", ["uniform", "clustered"])
def test_tabulated_interval_search_modes(pkg, orc, spacing):
    """Uniform knots take the kernels' binned interval search, knots
    clustered at one end (a cubic spacing) the binary search; both match the
    oracle, with queries on and next to the knots, at the bin edges and far
    outside the table.  The table holds a smooth function bounded away from
    zero, so every particle collapses and a wrong interval shows in F."""
    rng = np.random.default_rng(17)
    t = np.linspace(0.0, 1.0, 33)
    if spacing == "uniform":
        xk, yk, dk = 6.0 * t[:25], 6.0 * t[:21], -4.0 + 12.0 * t
    else:
        xk, yk, dk = 6.0 * t[:25] ** 3, 6.0 * t[:21] ** 3, -4.0 + 12.0 * t ** 3
    xk, yk = xk / xk[-1] * 6.0, yk / yk[-1] * 6.0
    sigma = 0.7
    X, Y, Dl = np.meshgrid(xk * sigma, yk * sigma, dk * sigma, indexing="ij")
    tab = orc.Table(xk * sigma, yk * sigma, dk * sigma,
                    1.5 + np.sin(1.3 * X + 0.4) * np.cos(0.7 * Y) + 0.05 * (Dl - 1.0) ** 2)
    pts = [rng.uniform(-1, 7, 3000), rng.uniform(-1, 7, 3000), rng.uniform(-6, 10, 3000)]
    for ax, k in enumerate((xk, yk, dk)):
        edges = k[0] + (k[-1] - k[0]) * np.arange(4 * (len(k) - 1) + 1) / (4 * (len(k) - 1))
        on = np.concatenate([k, edges, np.nextafter(k, -np.inf), np.nextafter(k, np.inf)])
        pts[ax] = np.concatenate([pts[ax], rng.permutation(np.resize(on, 3000))])
    pts = [np.concatenate([p, [-50.0, 50.0, 1e6]]) for p in pts]
    m = min(len(p) for p in pts)
    x, y, d = (p[:m] * sigma for p in pts)
    x, y = np.abs(x), np.abs(y)
    l2 = (d - x + y) / 3.0
    h6 = np.zeros((6, m))
    h6[0], h6[1], h6[2] = l2 + x, l2, l2 - y
    a, D = synth.growth_table(0.3)
    ref, got, _ = _run(pkg, orc, (xk, yk, dk), [h6], [sigma], a, D, tables=[tab])
    assert np.all(ref[0] > 0.4)
    compare(ref, got, label=f"interval search {spacing}")
