"""Shared test helpers: input preparation and parity comparison.

Inputs come from the seeded generator (synth); expected values come from the
oracle only.
"""

from __future__ import annotations

import numpy as np
import torch

import synth

REL_TOL = 1e-9   # relative tolerance on D_c = 1/Fmax and a_coll (plain FP64 path)


def c1_inputs(device="cpu"):
    cfg = synth.config("C1")
    slabs = [h for _, h in synth.hessian_slabs(cfg["n_side"], cfg["box"], cfg["radii"], cfg["seed"],
                                               cfg["cosmo"], device=device)]
    a, D = synth.growth_table(cfg["cosmo"].omega_m, cfg["n_growth"])
    return cfg, slabs, a, D


def run_gpu_radii(col, slabs, acoll=True, sigmas=None, tables=None, cosmo=0):
    """Apply every slab (6, n) device tensor in order; returns host arrays."""
    n = slabs[0].shape[1]
    Fmax, Rmax, ac = col.outputs(n)
    for r, h in enumerate(slabs):
        col.apply(h, r, Fmax, Rmax, ac if acoll else None, reset=(r == 0), cosmo=cosmo,
                  sigma_R=1.0 if sigmas is None else sigmas[r],
                  table_F=None if tables is None else tables[r])
    torch.cuda.synchronize()
    return Fmax.cpu().numpy(), Rmax.cpu().numpy(), (ac.cpu().numpy() if acoll else None)


def near_tie_mask(F_per_radius):
    """Particles whose two largest per-radius F are within 1e-12 relative."""
    Fs = np.sort(np.asarray(F_per_radius), axis=0)
    if Fs.shape[0] < 2:
        return np.zeros(Fs.shape[1], dtype=bool)
    top, second = Fs[-1], Fs[-2]
    return (top > 0) & (np.abs(top - second) <= 1e-12 * top)


def compare(ref, got, rel=REL_TOL, tie_mask=None, label=""):
    """ref/got: (Fmax, Rmax, acoll).  Returns a dict of statistics; asserts the
    parity gate: index exact (except near-ties), rel on D_c and a_coll for
    Fmax >= 1e-6, |dF| <= 1e-15 otherwise."""
    Fr, Rr, Ar = ref
    Fg, Rg, Ag = got
    big = Fr >= 1e-6
    both = big & (Fg > 0)
    assert np.array_equal(Fr > 0, Fg > 0) or np.all(np.abs(Fr - Fg)[(Fr > 0) != (Fg > 0)] <= 1e-15), \
        f"{label}: collapse/no-collapse sets differ"
    dD = np.abs(1.0 / Fg[both] - 1.0 / Fr[both]) * Fr[both] if both.any() else np.zeros(1)
    assert np.all(dD <= rel), f"{label}: max rel D_c err {dD.max():.3e}"
    small = ~big
    if small.any():
        assert np.max(np.abs(Fr[small] - Fg[small])) <= 1e-15, f"{label}: small-F mismatch"
    # a particle whose collapse decision flips within the 1e-15 allowance on F
    # (checked above) has no unique radius index
    mism = (Rr != Rg) & ((Fr > 0) == (Fg > 0))
    if tie_mask is not None:
        mism &= ~tie_mask
    assert not mism.any(), f"{label}: {int(mism.sum())} radius-index mismatches"
    stats = {"max_rel_D": float(dD.max()), "n": int(Fr.size), "collapsed": int(big.sum())}
    if Ar is not None and Ag is not None:
        fin = np.isfinite(Ar)
        assert np.array_equal(fin, np.isfinite(Ag)), f"{label}: a_coll finiteness differs"
        if fin.any():
            da = np.abs(Ag[fin] - Ar[fin]) / Ar[fin]
            assert np.all(da <= rel), f"{label}: max rel a_coll err {da.max():.3e}"
            stats["max_rel_a"] = float(da.max())
    return stats


EPS32 = 2.0 ** -24


def rel_stats(x):
    """max, p99.9 and mean of an array of relative errors."""
    x = np.asarray(x)
    if x.size == 0:
        return {"max": 0.0, "p99.9": 0.0, "mean": 0.0}
    return {"max": float(np.max(x)), "p99.9": float(np.percentile(x, 99.9)), "mean": float(np.mean(x))}


def mixed_bound(orc, slabs):
    """Per-particle tolerance on D_c of the mixed-precision path over the
    given radii (FP64 arrays (6, n)): D_c is homogeneous of degree -1 in the
    eigenvalues and the FP32 eigenvalue is off by a few eps32 |H|_F, so
    |dD_c/D_c| <= 64 eps32 |H|_F / l1; the max over radii is taken, since
    which radius wins is not known in advance.  Radii with l1 <= 0 give F = 0
    on both sides (no collapse) and add nothing; a particle with l1 <= 0 at
    every radius gets 0 (its F is 0 and never gated on D_c)."""
    b = None
    for h in slabs:
        lam, _ = orc.points(h)
        hn = np.sqrt(np.sum(h[:3] ** 2, axis=0) + 2 * np.sum(h[3:] ** 2, axis=0))
        pos = lam[:, 0] > 0
        br = np.zeros_like(hn)
        br[pos] = 64 * EPS32 * hn[pos] / lam[pos, 0]
        b = br if b is None else np.maximum(b, br)
    return b
