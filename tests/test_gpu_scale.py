"""The 512^3 x 40-radius configuration at full size (134M particles, one
GPU's share of a 2048^3 run), FP32 Hessians streamed one radius at a time,
through the mixed-precision path and through the surrogate + certify path
on the same fields.  The oracle recomputes a seeded sample of particles over
all 40 radii, both from the FP64 field (the error the mixed path is quoted
with) and from the FP32 inputs widened to FP64 (what the kernels read; the
gates).  Gates: mixed, the per-particle FP32 bound of the mixed tests;
surrogate, 1e-6 relative on D_c and a_coll after certification."""

import numpy as np
import pytest
import torch

import synth
from tests._helpers import EPS32, mixed_bound, rel_stats

pytestmark = pytest.mark.gpu


def test_512cube_40radii_mixed_and_surrogate(orc, trained_net):
    import paper_2510_02873_amd as P
    from paper_2510_02873_amd import _abi
    blob = trained_net[0]
    cfg = synth.config("C3")
    n_side, box, radii, cosmo = cfg["n_side"], cfg["box"], cfg["radii"], cfg["cosmo"]
    n = n_side ** 3
    a, D = synth.growth_table(cosmo.omega_m, cfg["n_growth"])
    sig = synth.grid_sigma_gauss(n_side, box, radii, cosmo, device="cuda")
    fld = synth.fields.field(n_side, box, cfg["seed"], cosmo, device="cuda")
    rng = np.random.default_rng(1234)
    idx = np.concatenate([np.sort(rng.choice(n, size=20000, replace=False)), [0, n - 1]])
    tidx = torch.from_numpy(idx).cuda()
    s64, s32 = [], []
    print(f"512^3 x {len(radii)}: n={n}", flush=True)
    with P.Collapse([(a, D, cosmo.omega_m)], precision=P.PINO_MIXED) as mix, \
            P.Collapse([(a, D, cosmo.omega_m)], precision=P.PINO_SURROGATE, mlp_blob=blob) as sur:
        Fm, Rm, Am = mix.outputs(n)
        Fs, Rs, As = sur.outputs(n)
        _abi.pino_collapse_surrogate_stats(sur.ctx, reset=True)
        last = len(radii) - 1
        for r, R in enumerate(radii):
            h64 = fld.hessian(R)
            s64.append(h64[:, tidx].cpu().numpy())
            h32 = h64.float()
            del h64
            s32.append(h32[:, tidx].double().cpu().numpy())
            mix.apply(h32, r, Fm, Rm, Am if r == last else None, reset=(r == 0), finalize=(r == last))
            sur.apply(h32, r, Fs, Rs, As if r == last else None, reset=(r == 0), finalize=(r == last),
                      sigma_R=sig[r])
            del h32
            if r % 10 == 9:
                torch.cuda.synchronize()
                print(f"  radius {r + 1}/{len(radii)} done", flush=True)
        torch.cuda.synchronize()
        stats = _abi.pino_collapse_surrogate_stats(sur.ctx)
        gm = [t[tidx].cpu().numpy() for t in (Fm, Rm, Am)]
        gs = [t[tidx].cpu().numpy() for t in (Fs, Rs, As)]
    g = orc.Growth(a, D)
    ref_w = orc.collapse(s32, g)
    ref_f = orc.collapse(s64, g)
    per_r = np.stack([orc.points(h)[1] for h in s32])
    srt = np.sort(per_r, axis=0)
    bound = mixed_bound(orc, s32)

    # mixed precision: report per output against both oracle runs, gate on
    # the same inputs
    for name, (Fr, Rr, Ar) in (("FP32 inputs", ref_w), ("FP64 field", ref_f)):
        big = Fr >= 1e-6
        rD = np.abs(1 / gm[0][big] - 1 / Fr[big]) * Fr[big]
        fin = np.isfinite(Ar) & np.isfinite(gm[2])
        ra = np.abs(gm[2][fin] - Ar[fin]) / Ar[fin]
        print(f"mixed vs oracle ({name}): D_c {rel_stats(rD)} a_coll {rel_stats(ra)} "
              f"index mismatches {int(np.sum(gm[1] != Rr))}/{Fr.size}", flush=True)
    Fr, Rr, Ar = ref_w
    big = Fr >= 1e-6
    rD = np.abs(1 / gm[0][big] - 1 / Fr[big]) * Fr[big]
    assert np.all(rD <= bound[big] + 1e-12)
    close = np.abs(srt[-1] - srt[-2]) <= 2 * bound * np.abs(srt[-1])
    assert np.all((gm[1] == Rr) | close)
    fin = np.isfinite(Ar)
    assert np.array_equal(fin, np.isfinite(gm[2]))
    assert np.all(np.abs(gm[2][fin] - Ar[fin]) / Ar[fin] <= (bound + 16 * EPS32)[fin])

    # surrogate + certify
    consulted = stats["certified"] + stats["fallback"]
    assert stats["certified"] + stats["fallback"] + stats["gated"] == n * len(radii)
    rD = np.abs(1 / gs[0][big] - 1 / Fr[big]) * Fr[big]
    ra = np.abs(gs[2][fin] - Ar[fin]) / Ar[fin]
    tie = np.abs(srt[-1] - srt[-2]) <= 2e-6 * srt[-1]
    print(f"surrogate 512^3 x 40: certified {stats['certified']} fallback {stats['fallback']} "
          f"gated {stats['gated']} (fallback fraction of consulted {stats['fallback'] / consulted:.3f}); "
          f"vs oracle (FP32 inputs): D_c {rel_stats(rD)} a_coll {rel_stats(ra)} "
          f"index mismatches {int(np.sum(gs[1] != Rr))}", flush=True)
    assert np.array_equal(gs[0] > 0, Fr > 0)
    assert rD.max() <= 1e-6 and ra.max() <= 1e-6
    assert np.array_equal(np.isfinite(gs[2]), fin)
    assert np.all((gs[1] == Rr) | tie)
