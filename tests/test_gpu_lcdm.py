"""GPU parity of the Classic method with flat-LCDM time coefficients
(PINO_CLASSIC_LCDM) against the oracle, through the C ABI.

The library integrates the growth ratios of the LPT terms on the device at
init (RK4 of the perturbation ODEs); the oracle computes them by a
Green's-function quadrature.  Gates: the ratios at the knots within 1e-9;
D_c = 1/Fmax and a_coll within 1e-9 relative, radius index exact except at
near-ties and where the oracle's root is nearly tangent (|dG/dln D| < 1e-6,
reported); Omega_m = 1 reproduces the Einstein-de Sitter Classic path."""

import numpy as np
import pytest
import torch

import synth
from tests._helpers import c1_inputs, compare, near_tie_mask, run_gpu_radii

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2510_02873_amd as P
    return P


@pytest.mark.parametrize("om,nk", [(0.3, 512), (0.27, 300), (1.0, 512), (0.35, 2048)])
def test_lpt_coefficients_vs_oracle(pkg, orc, om, nk):
    from paper_2510_02873_amd import _abi
    a, D = synth.growth_table(om, nk)
    with pkg.Collapse([(a, D, om)], method=pkg.PINO_CLASSIC_LCDM) as col:
        got = _abi.pino_collapse_lpt_coefficients(col.ctx, 0, nk)
    ref = orc.lpt_growth(om, a)
    worst = max(float(np.max(np.abs(g - r))) for g, r in zip(got, ref))
    print(f"Omega_m={om} nk={nk}: LCDM ratios at a=1 {[float(g[-1]) for g in got]}, max |GPU - oracle| "
          f"{worst:.2e}", flush=True)
    assert worst <= 1e-9


def test_lcdm_cosmologies_with_different_knot_counts(pkg, orc):
    """One context holding two cosmologies whose growth tables have different
    knot counts (300 and 512): the ratio rows of each are read with its own
    count (regression: rows laid out with the larger count were read with
    the smaller), so both the coefficients and the collapse of items of
    either cosmology match the oracle."""
    from paper_2510_02873_amd import _abi
    cfg, slabs, _, _ = c1_inputs()
    hs = [h.cuda() for h in slabs[:6]]
    tabs = [(0.35, 300), (0.27, 512)]
    growth = [(*synth.growth_table(om, nk), om) for om, nk in tabs]
    with pkg.Collapse(growth, method=pkg.PINO_CLASSIC_LCDM) as col:
        for k, (om, nk) in enumerate(tabs):
            got = _abi.pino_collapse_lpt_coefficients(col.ctx, k, nk)
            ref = orc.lpt_growth(om, growth[k][0])
            assert max(float(np.max(np.abs(g - r))) for g, r in zip(got, ref)) <= 1e-9
            res = run_gpu_radii(col, hs, cosmo=k)
            refc, skip, _ = _lcdm_ref(orc, hs, growth[k][0], growth[k][1], om)
            compare(refc, res, tie_mask=skip, label=f"LCDM cosmology {k} (Omega_m {om}, {nk} knots)")


def _lcdm_ref(orc, slabs, a, D, om):
    g = orc.Growth(a, D, om)
    host = [h.cpu().numpy() if torch.is_tensor(h) else np.asarray(h) for h in slabs]
    ref = orc.collapse(host, g, method=orc.CLASSIC_LCDM)
    # per radius F, for near-ties of the radius index, and the tangency of
    # the oracle's root at each particle's winning radius
    per_r = []
    for h in host:
        n = h.shape[1]
        Fr, Rr = np.zeros(n), np.full(n, -1, np.int32)
        orc.update_radius(h, 0, g, Fr, Rr, None, reset=True, method=orc.CLASSIC_LCDM)
        per_r.append(Fr)
    ties = near_tie_mask(per_r)
    F, R, _ = ref
    tang = np.zeros(F.size, dtype=bool)
    for i in np.nonzero(F > 0)[0]:
        lam = orc.eig3(host[R[i]][:, i])
        Dc = 1.0 / F[i]
        _, dG = orc.g_lcdm(lam, g, Dc)
        tang[i] = abs(dG) * Dc < 1e-6
    return ref, ties | tang, int(tang.sum())


def test_lcdm_c1_vs_oracle(pkg, orc):
    cfg, slabs, a, D = c1_inputs()
    om = cfg["cosmo"].omega_m
    ref, skip, n_tang = _lcdm_ref(orc, slabs, a, D, om)
    with pkg.Collapse([(a, D, om)], method=pkg.PINO_CLASSIC_LCDM) as col:
        got = run_gpu_radii(col, [h.cuda() for h in slabs])
    st = compare(ref, got, tie_mask=skip, label="C1 LCDM")
    with pkg.Collapse([(a, D, om)]) as col:
        eds = run_gpu_radii(col, [h.cuda() for h in slabs])
    big = (ref[0] > 1e-6) & (eds[0] > 0)
    shift = np.abs(ref[0][big] / eds[0][big] - 1)
    print(f"C1 LCDM vs oracle {st}; nearly tangent roots {n_tang}; F shift from the EdS coefficients: "
          f"median {np.median(shift):.2e} max {shift.max():.2e}", flush=True)
    assert np.median(shift) > 1e-5   # the coefficients do change the result


def test_lcdm_eds_equals_classic(pkg, orc):
    cfg, slabs, _, _ = c1_inputs()
    a, D = synth.growth_table(1.0)
    dev = [h.cuda() for h in slabs]
    with pkg.Collapse([(a, D, 1.0)], method=pkg.PINO_CLASSIC_LCDM) as col:
        F1, R1, A1 = run_gpu_radii(col, dev)
    with pkg.Collapse([(a, D, 1.0)]) as col:
        F0, R0, A0 = run_gpu_radii(col, dev)
    big = F0 > 1e-6
    rel = np.abs(F1[big] / F0[big] - 1)
    print(f"Omega_m = 1: LCDM vs Classic max rel {rel.max():.2e}", flush=True)
    assert np.array_equal(F1 > 0, F0 > 0) and rel.max() <= 1e-9
    assert np.array_equal(R1, R0)


@pytest.mark.parametrize("nk", [512, 2048])
def test_lcdm_special_and_ragged(pkg, orc, nk):
    """Diagonal, spherical, planar, repeated and zero spectra, NaN input, and
    item sizes that leave partial waves; collapse before the first growth
    knot (lambda_1 of 900-2000, D_c below D_0 = 1.3e-3) and after the last
    one, where the ratios are held at their end values.  512 knots read the
    ratio splines as power-form coefficients, 2048 as the (k, M) rows."""
    a, D = synth.growth_table(0.3, nk)
    rows = []
    for lam in [(1, 1, 1), (2, 0, 0), (1, 1, 0), (3, 3, -1), (0.5, -0.5, -0.5), (40.0, 3.0, -2.0), (-1, -2, -3),
                (0, 0, 0), (1e-3, 0, 0), (0.05, 0.01, -0.02), (8.0, 7.9, 7.8), (2000.0, 10.0, -5.0),
                (900.0, 899.0, 898.0), (1500.0, -700.0, -700.0)]:
        rows.append([lam[0], lam[1], lam[2], 0, 0, 0])
    rng = np.random.default_rng(8)
    rows += list(rng.normal(size=(300, 6)) * rng.uniform(0.1, 3.0, size=(300, 1)))
    H = np.ascontiguousarray(np.array(rows).T)
    g = orc.Growth(a, D, 0.3)
    for n in (1, 7, 64, 65, H.shape[1]):
        h = np.ascontiguousarray(H[:, :n])
        F = np.zeros(n)
        R = np.full(n, -1, np.int32)
        A = np.full(n, np.inf)
        orc.update_radius(h, 0, g, F, R, A, reset=True, method=orc.CLASSIC_LCDM)
        with pkg.Collapse([(a, D, 0.3)], method=pkg.PINO_CLASSIC_LCDM) as col:
            got = run_gpu_radii(col, [torch.from_numpy(h).cuda()])
        compare((F, R, A), got, label=f"LCDM special n={n} ({nk} knots)")
    # NaN never updates the maximum
    hn = np.full((6, 3), np.nan)
    with pkg.Collapse([(a, D, 0.3)], method=pkg.PINO_CLASSIC_LCDM) as col:
        Fg, Rg, _ = run_gpu_radii(col, [torch.from_numpy(hn).cuda()])
    assert np.all(Fg == 0) and np.all(Rg == -1)


@pytest.mark.parametrize("n", [1, 3, 1001])
def test_lcdm_unaligned_matches_aligned(pkg, orc, n):
    """Arrays 8- but not 16-byte aligned take the one-particle-per-lane LCDM
    kernel; its results equal the paired kernel's bit for bit (same
    arithmetic) and the oracle's.  Odd and tiny sizes exercise the paired
    kernel's last-element path."""
    cfg, slabs, a, D = c1_inputs()
    om = cfg["cosmo"].omega_m
    hs = [s[:, :n].contiguous() for s in slabs[:3]]
    with pkg.Collapse([(a, D, om)], method=pkg.PINO_CLASSIC_LCDM) as col:
        F1, R1, A1 = col.outputs(n)
        bufF = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        bufR = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        bufA = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        F2, R2, A2 = bufF[1:], bufR[1:], bufA[1:]
        last = len(hs) - 1
        for r, h in enumerate(hs):
            hd = h.cuda()
            buf = torch.empty((6, n + 1), dtype=torch.float64, device="cuda")
            buf[:, 1:] = hd
            hu = [buf[c, 1:] for c in range(6)]
            assert hu[0].data_ptr() % 16 == 8
            col.apply(hd, r, F1, R1, A1 if r == last else None, reset=(r == 0), finalize=(r == last))
            col.apply(hu, r, F2, R2, A2 if r == last else None, reset=(r == 0), finalize=(r == last))
        torch.cuda.synchronize()
        assert torch.equal(F1, F2) and torch.equal(R1, R2) and torch.equal(A1, A2)
    ref, skip, _ = _lcdm_ref(orc, hs, a, D, om)
    compare(ref, (F1.cpu().numpy(), R1.cpu().numpy(), A1.cpu().numpy()), tie_mask=skip,
            label=f"LCDM unaligned n={n}")


@pytest.mark.parametrize("nk", [1024, 2048])
def test_lcdm_large_tables_both_layouts(pkg, orc, nk):
    """The collapse kernels read the ratio splines as power-form coefficients
    per interval where those fit in LDS (1024 knots: about 139 KB) and as the
    (k, M) rows at the knots past that (2048 knots: the coefficients would
    need 254 KB, the rows need 156 KB).  Either way the paired and the
    one-per-lane kernels agree bit for bit and match the oracle on three C1
    radii."""
    cfg, slabs, _, _ = c1_inputs()
    om = cfg["cosmo"].omega_m
    a, D = synth.growth_table(om, nk)
    n = 4001
    hs = [s[:, :n].contiguous() for s in slabs[:3]]
    with pkg.Collapse([(a, D, om)], method=pkg.PINO_CLASSIC_LCDM) as col:
        F1, R1, A1 = col.outputs(n)
        bufF = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        bufR = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        bufA = torch.empty(n + 1, dtype=torch.float64, device="cuda")
        F2, R2, A2 = bufF[1:], bufR[1:], bufA[1:]
        last = len(hs) - 1
        for r, h in enumerate(hs):
            hd = h.cuda()
            buf = torch.empty((6, n + 1), dtype=torch.float64, device="cuda")
            buf[:, 1:] = hd
            hu = [buf[c, 1:] for c in range(6)]
            col.apply(hd, r, F1, R1, A1 if r == last else None, reset=(r == 0), finalize=(r == last))
            col.apply(hu, r, F2, R2, A2 if r == last else None, reset=(r == 0), finalize=(r == last))
        torch.cuda.synchronize()
        assert torch.equal(F1, F2) and torch.equal(R1, R2) and torch.equal(A1, A2)
    ref, skip, _ = _lcdm_ref(orc, hs, a, D, om)
    compare(ref, (F1.cpu().numpy(), R1.cpu().numpy(), A1.cpu().numpy()), tie_mask=skip,
            label=f"LCDM with {nk} growth knots")


def test_lcdm_unsupported_combinations(pkg):
    a, D = synth.growth_table(0.3)
    for kw in (dict(precision=pkg.PINO_MIXED),):
        with pytest.raises(pkg.PinoError) as e:
            pkg.Collapse([(a, D, 0.3)], method=pkg.PINO_CLASSIC_LCDM, **kw)
        assert e.value.status == pkg.PINO_ERR_UNSUPPORTED
    with pytest.raises(pkg.PinoError) as e:
        pkg.Collapse([(a, D, 1.5)], method=pkg.PINO_CLASSIC_LCDM)
    assert e.value.status == pkg.PINO_ERR_ARG
