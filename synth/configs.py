"""The workloads, as plain data.

C1  plain FP64, 32^3 in a periodic 100 Mpc/h box, 4 Gaussian radii 8..1 Mpc/h,
    512-point growth table with a in [1e-3, 1].
C2  plain FP64, 256^3 (same box), 25 radii 20..0.5 Mpc/h, each radius a
    separate SoA FP64 slab.
C3  mixed precision, 512^3 in 200 Mpc/h (same cell size as C2), 40 radii
    20..0.5 Mpc/h, FP32 slabs plus FP64 copies for the degenerate branch.
C4  batched: 64 realisations, grid side uniform in {64..192}, cell 0.78125
    Mpc/h, Omega_m ~ U[0.25, 0.35], sigma8 ~ U[0.7, 0.9], 20 radii 16..1 Mpc/h.
C5  surrogate at 512^3 x 40 radii (as C3).
C2T the C2 fields through the tabulated kernel with a 64 x 64 x 128 table.

Radii are processed from large to small (reading; the paper does not state the
order).  Flat LCDM Omega_m = 0.3, sigma8 = 0.8, n_s = 0.96, h = 0.7, BBKS.
"""

from __future__ import annotations

import numpy as np

from .cosmo import Cosmology
from .fields import log_radii

BASE = Cosmology(omega_m=0.3, sigma8=0.8, n_s=0.96)

CONFIGS = {
    "C1": dict(name="plain-fp64-32cube-4radii", n_side=32, box=100.0, seed=1,
               radii=log_radii(8.0, 1.0, 4), n_growth=512, cosmo=BASE, precision="fp64"),
    "C2": dict(name="plain-fp64-256cube-25radii", n_side=256, box=100.0, seed=2,
               radii=log_radii(20.0, 0.5, 25), n_growth=512, cosmo=BASE, precision="fp64"),
    "C3": dict(name="mixed-512cube-40radii", n_side=512, box=200.0, seed=3,
               radii=log_radii(20.0, 0.5, 40), n_growth=512, cosmo=BASE, precision="mixed"),
    "C5": dict(name="surrogate-512cube-40radii", n_side=512, box=200.0, seed=3,
               radii=log_radii(20.0, 0.5, 40), n_growth=512, cosmo=BASE, precision="surrogate"),
    "C2T": dict(name="tabulated-fp64-256cube-25radii", n_side=256, box=100.0, seed=2,
                radii=log_radii(20.0, 0.5, 25), n_growth=512, cosmo=BASE, precision="fp64",
                table=(64, 64, 128)),
}


def batched_realisations(master_seed: int = 4, count: int = 64, n_min: int = 64, n_max: int = 192,
                         cell: float = 0.78125):
    """C4: per-realisation (n_side, box, seed, Cosmology), drawn from master_seed."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    out = []
    for r in range(count):
        n_side = int(rng.integers(n_min, n_max + 1))
        om = float(rng.uniform(0.25, 0.35))
        s8 = float(rng.uniform(0.7, 0.9))
        out.append(dict(n_side=n_side, box=n_side * cell, seed=1000 * master_seed + r,
                        cosmo=Cosmology(omega_m=om, sigma8=s8, n_s=0.96)))
    return out


CONFIGS["C4"] = dict(name="batched-64real-20radii", realisations=batched_realisations(),
                     radii=log_radii(16.0, 1.0, 20), n_growth=512, precision="fp64")


def config(key: str) -> dict:
    return CONFIGS[key]
