"""Mixed-precision paths against the FP64 oracle.  Classic: FP32 Hessians
and eigenvalues, FP64 root polish and nearly-repeated branch, FP32 growth
interpolation.  Tabulated: FP32 Hessians, FP32 eigenvalues (FP64 for nearly
repeated pairs), FP32 cell search and interpolation on an FP32 copy of the
table, gated per particle by the bound derived in _tab32_bound.

The oracle runs on the same inputs the kernel reads (the FP32 Hessians
widened to FP64), which isolates the arithmetic error, and on the original
FP64 field, which adds the input rounding; both are reported per output.
Gate, derived from FP32 rounding (eps = 2^-24): the FP32 eigenvalue is off by
a few eps * |H|, and D_c is homogeneous of degree -1 in the eigenvalues, so
per particle |dD_c/D_c| <= 64 eps |H|_F / l1; the FP32 spline adds a few eps
to a_coll."""

import numpy as np
import pytest
import torch

import synth
from tests._helpers import EPS32, c1_inputs, mixed_bound, rel_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2510_02873_amd as P
    return P


def _rel(a, b):
    return np.abs(a - b) / np.abs(b)


_stats = rel_stats


def _bound(orc, slabs32):
    return mixed_bound(orc, slabs32)


def test_mixed_c1(pkg, orc):
    cfg, slabs, a, D = c1_inputs()
    slabs32 = [h.to(torch.float32) for h in slabs]
    widened = [h.to(torch.float64).numpy() for h in slabs32]
    g = orc.Growth(a, D)
    ref_w = orc.collapse(widened, g)
    ref_f = orc.collapse([h.numpy() for h in slabs], g)
    with pkg.Collapse([(a, D)], precision=pkg.PINO_MIXED) as col:
        n = slabs[0].shape[1]
        Fm, Rm, ac = col.outputs(n)
        last = len(slabs32) - 1
        for r, h in enumerate(slabs32):
            col.apply(h.cuda().contiguous(), r, Fm, Rm, ac if r == last else None, reset=(r == 0),
                      finalize=(r == last))
        torch.cuda.synchronize()
        F, R, A = Fm.cpu().numpy(), Rm.cpu().numpy(), ac.cpu().numpy()
    bound = _bound(orc, widened)
    for name, (Fr, Rr, Ar) in (("same inputs", ref_w), ("FP64 field", ref_f)):
        big = Fr >= 1e-6
        rD = _rel(1 / F[big], 1 / Fr[big])
        fin = np.isfinite(Ar) & np.isfinite(A)
        ra = _rel(A[fin], Ar[fin])
        print(f"mixed vs oracle ({name}): D_c {_stats(rD)}  a_coll {_stats(ra)}  "
              f"index mismatches {int(np.sum(R != Rr))}/{n}", flush=True)
    Fr, Rr, Ar = ref_w
    big = Fr >= 1e-6
    rD = _rel(1 / F[big], 1 / Fr[big])
    assert np.all(rD <= bound[big] + 1e-12), f"worst excess {np.max(rD - bound[big]):.3e}"
    # radius index: exact unless the top two radii are within the FP32 bound
    per_r = np.stack([orc.points(h)[1] for h in widened])
    srt = np.sort(per_r, axis=0)
    close = np.abs(srt[-1] - srt[-2]) <= 2 * bound * np.abs(srt[-1])
    assert np.all((R == Rr) | close)
    fin = np.isfinite(Ar)
    assert np.array_equal(fin, np.isfinite(A))
    tol_a = bound + 16 * EPS32
    assert np.all(_rel(A[fin], Ar[fin]) <= tol_a[fin])


def test_mixed_special_and_ragged(pkg, orc):
    from tests.test_gpu_classic import _special_hessians
    a, D = synth.growth_table(0.3)
    rng = np.random.default_rng(2)
    for h6 in (_special_hessians(), rng.normal(size=(6, 4097)) * 0.7):
        h32 = torch.from_numpy(h6).to(torch.float32)
        wid = h32.to(torch.float64).numpy()
        n = wid.shape[1]
        F0, R0, A0 = np.zeros(n), np.full(n, -1, np.int32), np.full(n, np.inf)
        orc.update_radius(wid, 0, orc.Growth(a, D), F0, R0, A0, reset=True)
        with pkg.Collapse([(a, D)], precision=pkg.PINO_MIXED) as col:
            Fm, Rm, ac = col.outputs(n)
            col.apply(h32.cuda().contiguous(), 0, Fm, Rm, ac, reset=True, sync=True)
            F, R, A = Fm.cpu().numpy(), Rm.cpu().numpy(), ac.cpu().numpy()
        bound = _bound(orc, [wid])
        assert np.array_equal(F > 0, F0 > 0)
        big = F0 >= 1e-6
        assert np.all(_rel(1 / F[big], 1 / F0[big]) <= bound[big] + 1e-12)
        assert np.array_equal(R, R0)


def _table_lipschitz(t):
    """Bounds on |dF/dx|, |dF/dy| and |dF/ddelta| of the interpolant of one
    oracle table (knots in the kernel's units).  Along delta each row is a
    natural spline: on [d_i, d_i+1], S' = slope_i + h/6 ((1 - 3A^2) M_i +
    (3B^2 - 1) M_i+1) with A + B = 1 in [0, 1], so |S'| <= |slope_i| +
    h/3 (|M_i| + |M_i+1|).  Across x (and y) the interpolant is linear in the
    corner rows; the difference of two rows is the natural spline of the
    differences, whose piece is the chord plus h^2/6 ((A^3 - A) dM_i +
    (B^3 - B) dM_i+1), |A^3 - A| <= 0.385, so sup|S_b - S_a| over an interval
    <= max(|dF_i|, |dF_i+1|) + 0.0642 h^2 (|dM_i| + |dM_i+1|)."""
    F, M = t.F, t.M
    h = np.diff(t.dk)

    def row_diff_sup(dF, dM):
        a = np.maximum(np.abs(dF[..., :-1]), np.abs(dF[..., 1:]))
        return np.max(a + 0.0642 * h * h * (np.abs(dM[..., :-1]) + np.abs(dM[..., 1:])))

    Lx = max(row_diff_sup(F[i + 1] - F[i], M[i + 1] - M[i]) / (t.xk[i + 1] - t.xk[i])
             for i in range(len(t.xk) - 1))
    Ly = max(row_diff_sup(F[:, j + 1] - F[:, j], M[:, j + 1] - M[:, j]) / (t.yk[j + 1] - t.yk[j])
             for j in range(len(t.yk) - 1))
    slope = np.diff(F, axis=2) / h
    Ld = np.max(np.abs(slope) + h / 3 * (np.abs(M[..., :-1]) + np.abs(M[..., 1:])))
    return Lx, Ly, Ld


def _tab32_bound(orc, tables, slabs):
    """Per-particle bound on |F_mixed - F_oracle| (the oracle on the FP32
    inputs widened to FP64), the maximum over radii of (the maximum is
    1-Lipschitz):
      - the table rounded to FP32: the interpolant is linear in the table
        values with weights (1 - t), t and h^2/6 ((1-t)^3 - (1-t)) etc.
        (|.| <= 0.385 h^2/6) inside convex bilinear weights, so
        eps (max|F| + 0.1284 h^2 max|M|);
      - the FP32 spline and bilinear arithmetic: a few roundings of terms of
        that size, taken as 10 eps (max|F| + 0.1284 h^2 max|M|);
      - the cell coordinates: each FP32 eigenvalue is within 64 eps |H|_F
        outside the nearly repeated band (the FP64 path decides inside it;
        a host build of the same FP32 code reaches 44 eps |H|_F on 2.4M
        matrices with gaps down to 1e-4 of the scale), so x = l1 - l2 and
        y = l2 - l3 move by <= 128 eps |H|_F, rounded to FP32 within
        another 4 eps |H|_F and 2 eps |H|_F of FP32 trace; the FP32 knots
        and the cell fractions add 4 eps max|knot| per axis; each moves F by
        the axis' Lipschitz bound (_table_lipschitz) times the shift."""
    b = None
    for h, t in zip(slabs, tables):
        h = np.asarray(h, dtype=np.float64)
        with np.errstate(invalid="ignore", over="ignore"):
            hn = np.sqrt(np.sum(h[:3] ** 2, axis=0) + 2 * np.sum(h[3:] ** 2, axis=0))
        hn[~np.isfinite(hn)] = 0.0   # non-finite input: F = 0 on both sides
        hmax = np.max(np.diff(t.dk))
        base = 11 * EPS32 * (np.max(np.abs(t.F)) + 0.1284 * hmax * hmax * np.max(np.abs(t.M)))
        Lx, Ly, Ld = _table_lipschitz(t)
        dx = 132 * EPS32 * hn + 4 * EPS32 * np.max(np.abs(t.xk))
        dy = 132 * EPS32 * hn + 4 * EPS32 * np.max(np.abs(t.yk))
        dd = 4 * EPS32 * hn + 4 * EPS32 * np.max(np.abs(t.dk))
        br = 1.01 * (base + Lx * dx + Ly * dy + Ld * dd)
        b = br if b is None else np.maximum(b, br)
    return b


def _mixed_tab_run(pkg, orc, knots, slabs32, sigmas, a, D, col_kw=None):
    """Oracle Tabulated on the FP32 Hessians widened to FP64 (FP64 tables)
    and the mixed-precision GPU path on the FP32 Hessians."""
    from tests.test_gpu_tabulated import _filled_table
    tabs = [_filled_table(orc, knots, s) for s in sigmas]
    widened = [h.to(torch.float64).numpy() for h in slabs32]
    g = orc.Growth(a, D)
    ref = orc.collapse(widened, g, method=orc.TABULATED, tables=tabs)
    per_r = []
    for h, t in zip(widened, tabs):
        n = h.shape[1]
        F, R, A = np.zeros(n), np.full(n, -1, np.int32), np.full(n, np.inf)
        orc.update_radius(h, 0, g, F, R, A, reset=True, method=orc.TABULATED, table=t)
        per_r.append(F)
    with pkg.Collapse([(a, D)], method=pkg.PINO_TABULATED, precision=pkg.PINO_MIXED, table_knots=knots,
                      **(col_kw or {})) as col:
        n = slabs32[0].shape[1]
        Fm, Rm, ac = col.outputs(n)
        last = len(slabs32) - 1
        for r, (h, t, s) in enumerate(zip(slabs32, tabs, sigmas)):
            tF = torch.from_numpy(np.ascontiguousarray(t.F)).cuda()
            col.apply(h.cuda().contiguous(), r, Fm, Rm, ac if r == last else None, reset=(r == 0),
                      finalize=(r == last), sigma_R=s, table_F=tF)
        torch.cuda.synchronize()
        got = (Fm.cpu().numpy(), Rm.cpu().numpy(), ac.cpu().numpy())
    return ref, got, np.stack(per_r), _tab32_bound(orc, tabs, widened)


def _check_mixed_tab(ref, got, per_r, b, label):
    Fr, Rr, Ar = ref
    F, R, A = got
    b = np.broadcast_to(np.asarray(b, dtype=np.float64), Fr.shape)
    dF = np.abs(F - Fr)
    print(f"{label}: |dF| max {dF.max():.2e} (bound: median {np.median(b):.2e}, min {np.min(b):.2e}; "
          f"largest |dF|/bound {np.max(dF / b):.3f}), index mismatches {int(np.sum(R != Rr))}", flush=True)
    assert np.all(dF <= b + 1e-12 * np.abs(Fr)), f"{label}: worst excess {np.max(dF - b):.3e}"
    # radius index: exact unless the top two radii are within the bound (or F ~ 0)
    srt = np.sort(per_r, axis=0)
    second = srt[-2] if srt.shape[0] > 1 else np.zeros_like(srt[-1])
    close = (np.abs(srt[-1] - second) <= 2 * b) | (np.abs(Fr) <= b)
    assert np.all((R == Rr) | close)
    fin = np.isfinite(Ar) & np.isfinite(A)
    odd = np.isfinite(Ar) != np.isfinite(A)
    assert np.all(np.abs(Fr[odd]) <= b[odd])
    big = fin & (Fr > 1e3 * b)
    ra = np.abs(A[big] - Ar[big]) / Ar[big]
    tol = b[big] / Fr[big] + 16 * EPS32
    assert np.all(ra <= tol), f"{label}: a_coll worst excess {np.max(ra - tol):.3e}"


def test_mixed_tabulated_c1(pkg, orc):
    """Mixed-precision Tabulated at C1 (32^3 x 4 radii, 64 x 64 x 128 tables):
    against the oracle on the same (FP32) inputs, F within the bound set by
    the FP32 table, radius index exact outside near-ties, a_coll within that
    bound plus the FP32 spline."""
    cfg, slabs, a, D = c1_inputs()
    slabs32 = [h.to(torch.float32) for h in slabs]
    sigmas = [synth.grid_sigma_gauss(cfg["n_side"], cfg["box"], R) for R in cfg["radii"]]
    knots = synth.table_knots(1.0, 64, 64, 128)
    ref, got, per_r, b = _mixed_tab_run(pkg, orc, knots, slabs32, sigmas, a, D)
    _check_mixed_tab(ref, got, per_r, b, "mixed tabulated C1")


def test_mixed_tabulated_special_and_ragged(pkg, orc):
    from tests.test_gpu_classic import _special_hessians
    a, D = synth.growth_table(0.3)
    rng = np.random.default_rng(4)
    knots = synth.table_knots(1.0, 16, 12, 40)
    for h6 in (_special_hessians(), rng.normal(size=(6, 4097)) * 0.7, rng.normal(size=(6, 1)) * 0.7):
        h32 = torch.from_numpy(h6).to(torch.float32)
        ref, got, per_r, b = _mixed_tab_run(pkg, orc, knots, [h32], [0.9], a, D)
        _check_mixed_tab(ref, got, per_r, b, f"mixed tabulated n={h6.shape[1]}")


@pytest.mark.parametrize("n", [1, 3, 1001])
def test_mixed_tabulated_unaligned_matches_aligned(pkg, orc, n):
    """FP32 components 4- but not 8-byte aligned take the one-particle-per-
    lane kernel; it equals the paired kernel bit for bit."""
    from tests.test_gpu_tabulated import _filled_table
    rng = np.random.default_rng(n + 11)
    knots = synth.table_knots(1.0, 16, 12, 40)
    a, D = synth.growth_table(0.3)
    tF = torch.from_numpy(np.ascontiguousarray(_filled_table(orc, knots, 0.8).F)).cuda()
    slabs = [torch.from_numpy(rng.normal(size=(6, n)) * 0.8).to(torch.float32).cuda() for _ in range(2)]
    with pkg.Collapse([(a, D)], method=pkg.PINO_TABULATED, precision=pkg.PINO_MIXED, table_knots=knots) as col:
        F1, R1, A1 = col.outputs(n)
        F2, R2, A2 = col.outputs(n)
        for r, hd in enumerate(slabs):
            buf = torch.empty((6, n + 1), dtype=torch.float32, device="cuda")
            buf[:, 1:] = hd
            hu = [buf[c, 1:] for c in range(6)]
            assert hu[0].data_ptr() % 8 == 4
            col.apply(hd, r, F1, R1, A1 if r == 1 else None, reset=(r == 0), finalize=(r == 1), sigma_R=0.8,
                      table_F=tF)
            col.apply(hu, r, F2, R2, A2 if r == 1 else None, reset=(r == 0), finalize=(r == 1), sigma_R=0.8,
                      table_F=tF)
        torch.cuda.synchronize()
        assert torch.equal(F1, F2) and torch.equal(R1, R2) and torch.equal(A1, A2)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 1001])
def test_mixed_unaligned_arrays_match_aligned(pkg, n):
    """FP32 components that are 4- but not 8-byte aligned take the
    one-particle-per-lane kernel; it equals the paired kernel bit for bit.
    Odd and tiny sizes exercise the paired kernel's last element."""
    cfg, slabs, a, D = c1_inputs()
    hs = [s[:, :n].to(torch.float32).contiguous() for s in slabs]
    with pkg.Collapse([(a, D)], precision=pkg.PINO_MIXED) as col:
        F1, R1, A1 = col.outputs(n)
        F2, R2, A2 = col.outputs(n)
        last = len(hs) - 1
        for r, h in enumerate(hs):
            hd = h.cuda()
            buf = torch.empty((6, n + 1), dtype=torch.float32, device="cuda")
            buf[:, 1:] = hd
            hu = [buf[c, 1:] for c in range(6)]
            assert hu[0].data_ptr() % 8 == 4
            col.apply(hd, r, F1, R1, A1 if r == last else None, reset=(r == 0), finalize=(r == last))
            col.apply(hu, r, F2, R2, A2 if r == last else None, reset=(r == 0), finalize=(r == last))
        torch.cuda.synchronize()
        assert torch.equal(F1, F2) and torch.equal(R1, R2) and torch.equal(A1, A2)
