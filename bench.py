#!/usr/bin/env python3
"""Benchmark of the collapse-time path on one MI355X.

Workload: 256^3 particles in a periodic 100 Mpc/h box, 25 Gaussian smoothing
radii log-spaced 20 -> 0.5 Mpc/h (flat LCDM, Omega_m = 0.3, sigma8 = 0.8,
n_s = 0.96, BBKS), 512-point growth table; plain FP64 Classic collapse.  All 25
FP64 Hessian slabs (20 GB) are resident in HBM before timing starts.  One
step = all 25 radii over all particles (one kernel launch per radius), i.e.
4.19e8 particle-radius collapse evaluations.

Prints one JSON line (rank 0): evals/s, the roofline of the collapse kernel
(algorithmic bytes per launch / its mean launch time from HIP events on the
launch stream) and the oracle's rate on a bounded sample of the same
workload on the host cores.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle·radius collapse evals/s, plain FP64 vs surrogate+certify, at ≤1e-6 rel err"
PROFILE = os.path.join(ROOT, "profiles", "k_classic_f64_256cube_25radii.txt")
HBM_PEAK_GBS = 8000.0
# surrogate training budget: 160k steps of 16384 pairs (about 130 epochs of
# the 20M pairs, ~8 s) certify ~93 % of consulted particles, against ~84 %
# after 40k steps and ~55 % after 10k
TRAIN_STEPS = 160000
FP64_PEAK_TFS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n, updates, reset, finalize, hess_bytes=48):
    """HBM bytes one launch must move: 6 Hessian components (48 B in FP64,
    24 B in FP32), the running Fmax (8 B, not read on the RESET radius),
    Fmax + Rmax (12 B) for every particle whose maximum changes (all of them
    on RESET), and a_coll (8 B per particle) on the finalizing launch."""
    b = n * hess_bytes + (0 if reset else n * 8) + (n if reset else updates) * 12
    return b + (n * 8 if finalize else 0)


def step_roofline(bytes_per_step, ms):
    """HBM roofline of a leg from its algorithmic bytes per step and its
    measured time per step (launch gaps included, so a lower bound)."""
    gbs = bytes_per_step / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_step": int(bytes_per_step)}


def _time_steps(step, steps, stream):
    import torch
    step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def measure_extras(P, col, slabs, radii, n, a, D, cfg, n_side, stream, Fmax, Rmax, ac, steps, dk=None,
                   updates=None, train_steps=TRAIN_STEPS, plain_ms=None, blob_path=None, blob_out=None):
    """Secondary rates on the same resident fields: mixed precision (FP32
    copies of the Hessians) and the Tabulated method (64 x 64 x 128 tables
    filled per radius by the library's Classic kernel on the table's sample
    points).  Each reports evals/s and the agreement of its outputs with the
    plain FP64 run just timed."""
    import numpy as np
    import torch

    import synth

    out = {}
    last = len(radii) - 1
    F64, R64, A64 = Fmax.clone(), Rmax.clone(), ac.clone()
    ups = updates or [n] * len(radii)

    def step_bytes(hess_bytes):
        return sum(algorithmic_bytes(n, u, r == 0, r == last, hess_bytes) for r, u in enumerate(ups))

    sig = synth.grid_sigma_gauss(n_side, cfg["box"], radii)

    # mixed precision
    s32 = [h.to(torch.float32) for h in slabs]
    mcol = P.Collapse([(a, D)], precision=P.PINO_MIXED)
    Fm, Rm, Am = mcol.outputs(n)
    mitems = [mcol.item(s32[r], Fm, Rm, Am if r == last else None, radius_index=r) for r in range(len(radii))]

    def mstep():
        for r, it in enumerate(mitems):
            mcol.eval([it], reset=(r == 0), finalize=(r == last), stream=stream)

    ms = _time_steps(mstep, steps, stream)
    big = F64 > 1e-6
    rel = ((1 / Fm[big] - 1 / F64[big]).abs() * F64[big]).cpu().numpy()
    out["mixed"] = {"value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s", "ms_per_step": round(ms, 4),
                    "dtype": "f32 inputs/eigen/interp, f64 root", "workload": f"same {n_side}^3 x {len(radii)} fields",
                    "rel_Dc_vs_fp64": {"max": float(rel.max()), "p99.9": float(np.percentile(rel, 99.9)),
                                       "mean": float(rel.mean())},
                    "index_mismatch_frac": float((Rm != R64).double().mean().item()),
                    "roofline": step_roofline(step_bytes(24), ms)}
    mcol.close()

    # the same FP64 workload through the batched persistent launch: the 25
    # radii are resident anyway, so one launch per step carries each particle
    # through all of them with the running maximum in registers (48 B per
    # evaluation plus 20 B per particle); its outputs must equal the
    # per-radius evals' bit for bit
    try:
        from paper_2510_02873_amd import _abi
        Fb, Rb, Ab = col.outputs(n)
        bat = _abi.Batch(col.ctx, [{"h": slabs, "Fmax": Fb, "Rmax": Rb, "a_coll": Ab, "cosmo": 0}],
                         flags=P.PINO_EVAL_RESET | P.PINO_EVAL_FINALIZE, autotune=True)
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            ms = _time_steps(lambda: bat.graph_launch(gs), steps, gs)
        out["batched_same_fields"] = {
            "value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s", "ms_per_step": round(ms, 4),
            "dtype": "f64", "workload": f"same {n_side}^3 x {len(radii)} fields, all radii resident",
            "launch": "one persistent kernel per step, HIP graph replay", "autotuned": bat.config(),
            "identical_to_per_radius": bool(torch.equal(Fb, F64) and torch.equal(Rb, R64) and torch.equal(Ab, A64)),
            "vs_per_radius_throughput": round(plain_ms / ms, 4) if plain_ms else None,
            "roofline": step_roofline(n * (48 * len(radii) + 20), ms)}
        bat.close()
        del Fb, Rb, Ab
    except RuntimeError as e:
        out["batched_same_fields"] = {"error": str(e)[:300]}

    out["surrogate"] = measure_surrogate(P, slabs, radii, sig, n, a, D, cfg, n_side, stream, F64, R64, steps,
                                         train_steps, blob_path, blob_out)
    out["_blob"] = out["surrogate"].pop("blob")
    # stream floor: FP64 Hessians once per particle (the deferred particles'
    # second read by the block's tail is not counted)
    out["surrogate"]["roofline"] = step_roofline(step_bytes(48), out["surrogate"]["ms_per_step"])
    out["surrogate"]["vs_plain_fp64_throughput"] = round(out["surrogate"]["value"] / (n * len(radii) / (
        plain_ms * 1e-3)), 4) if plain_ms else None

    # Tabulated: fill each radius' table with the Classic kernel on the
    # table's sample points (diagonal Hessians), then interpolate
    knots = synth.table_knots(1.0, 64, 64, 128)
    tabs = []
    for sR in sig:
        grid = torch.from_numpy(synth.table_grid_hessians(*(np.asarray(k) * sR for k in knots))).cuda()
        Ft, Rt, _ = col.outputs(grid.shape[1])
        col.apply(grid, 0, Ft, Rt, None, reset=True, stream=stream)
        tabs.append(Ft)
    tcol = P.Collapse([(a, D)], method=P.PINO_TABULATED, table_knots=knots)
    Ft, Rt, At = tcol.outputs(n)
    titems = [tcol.item(slabs[r], Ft, Rt, At if r == last else None, radius_index=r, sigma_R=sig[r],
                        table_F=tabs[r]) for r in range(len(radii))]

    def tstep():
        for r, it in enumerate(titems):
            tcol.eval([it], reset=(r == 0), finalize=(r == last), stream=stream)

    ms = _time_steps(tstep, steps, stream)
    both = (F64 > 0.05) & (Ft > 0)
    relt = ((Ft[both] - F64[both]).abs() / F64[both]).cpu().numpy()
    out["tabulated"] = {"value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s",
                        "ms_per_step": round(ms, 4), "table": "64x64x128 per radius, rebuilt on device",
                        "rel_F_vs_classic_median": float(np.median(relt)),
                        "roofline": step_roofline(step_bytes(48), ms),
                        "roofline_note": "HBM streams only; the corner gathers (128 B per evaluation) are served "
                                         "from L2/MALL (8.4 MB table)"}
    tcol.close()

    # Tabulated in mixed precision: FP32 Hessians, FP32 eigenvalues (FP64 for
    # nearly repeated pairs), FP32 cell search and interpolation on the FP32
    # knot-pair table (four 16-byte corner reads per evaluation)
    mtcol = P.Collapse([(a, D)], method=P.PINO_TABULATED, precision=P.PINO_MIXED, table_knots=knots)
    Fq, Rq, Aq = mtcol.outputs(n)
    qitems = [mtcol.item(s32[r], Fq, Rq, Aq if r == last else None, radius_index=r, sigma_R=sig[r],
                         table_F=tabs[r]) for r in range(len(radii))]

    def qstep():
        for r, it in enumerate(qitems):
            mtcol.eval([it], reset=(r == 0), finalize=(r == last), stream=stream)

    ms = _time_steps(qstep, steps, stream)
    relq = ((Fq[both] - Ft[both]).abs() / Ft[both]).cpu().numpy()
    out["tabulated_mixed"] = {"value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s",
                              "ms_per_step": round(ms, 4),
                              "dtype": "f32 inputs, eigenvalues, search, interpolation and table; f64 for nearly "
                                       "repeated pairs",
                              "rel_F_vs_fp64_tabulated": {"max": float(relq.max()),
                                                          "p99.9": float(np.percentile(relq, 99.9)),
                                                          "mean": float(relq.mean())},
                              "index_mismatch_frac": float((Rq != Rt).double().mean().item()),
                              "roofline": step_roofline(step_bytes(24), ms),
                              "roofline_note": "HBM streams only; the corner gathers (64 B per evaluation) are "
                                               "served from L2/MALL"}
    mtcol.close()
    del s32

    # Tabulated table from the homogeneous-ellipsoid integration: one
    # 64 x 64 x 128 table (524288 nodes) per radius; time the fill at the
    # smallest and the largest sigma
    from paper_2510_02873_amd import _abi
    ecol = P.Collapse([(a, D, cfg["cosmo"].omega_m)], method=P.PINO_TABULATED, table_knots=knots)
    Fe = torch.empty(64 * 64 * 128, dtype=torch.float64, device=slabs[0].device)
    fills = {}
    for r in (0, len(radii) - 1):
        _abi.pino_collapse_ellipsoid_table(ecol.ctx, 0, sig[r], Fe, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _abi.pino_collapse_ellipsoid_table(ecol.ctx, 0, sig[r], Fe, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        fills[f"sigma_{sig[r]:.3f}"] = round(e0.elapsed_time(e1), 3)
    frac_collapsing = float((Fe > 0).double().mean().item())
    ecol.close()
    out["ellipsoid_table"] = {"nodes": 64 * 64 * 128, "fill_ms": fills,
                              "collapsing_fraction_at_last_sigma": round(frac_collapsing, 4),
                              "method": "homogeneous ellipsoid, nine ODEs, RK4 (h = 0.01 in ln a), one thread "
                                        "per node"}
    log(f"ellipsoid table fill (64x64x128): {fills} ms")

    # Classic with flat-LCDM LPT time coefficients on the same FP64 fields
    lcol = P.Collapse([(a, D, cfg["cosmo"].omega_m)], method=P.PINO_CLASSIC_LCDM)
    Fl, Rl, Al = lcol.outputs(n)
    litems = [lcol.item(slabs[r], Fl, Rl, Al if r == last else None, radius_index=r) for r in range(len(radii))]

    def lstep():
        for r, it in enumerate(litems):
            lcol.eval([it], reset=(r == 0), finalize=(r == last), stream=stream)

    ms = _time_steps(lstep, steps, stream)
    bothl = (F64 > 1e-6) & (Fl > 0)
    shift = (Fl[bothl] / F64[bothl] - 1).abs().cpu().numpy()
    out["classic_lcdm"] = {"value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s",
                           "ms_per_step": round(ms, 4), "dtype": "f64",
                           "F_shift_vs_eds_coefficients": {"median": float(np.median(shift)),
                                                           "max": float(shift.max())},
                           "roofline": step_roofline(step_bytes(48), ms)}
    lcol.close()
    lcdm_ms = ms

    # the surrogate on the LCDM condition: network trained on LCDM targets of
    # the five cosmologies (its Omega_m input now matters), LCDM certificate
    # and full solve, against the plain LCDM run on the same fields
    sl = measure_surrogate(P, slabs, radii, sig, n, a, D, cfg, n_side, stream, Fl, Rl, steps, train_steps,
                           method=P.PINO_CLASSIC_LCDM)
    sl.pop("blob")
    sl["roofline"] = step_roofline(step_bytes(48), sl["ms_per_step"])
    sl["vs_plain_lcdm_throughput"] = round(lcdm_ms / sl["ms_per_step"], 4)
    out["surrogate_lcdm"] = sl
    del Fl, Rl, Al

    if dk is not None:
        out["field_fused"] = measure_field(P, col, dk, radii, n, n_side, cfg, stream, F64, R64, steps, [(a, D)])
    out["interp_sweep"] = measure_interp()
    return out


def _stats_ms(ts):
    import numpy as np
    ts = np.asarray(ts)
    return {"mean": round(float(ts.mean()), 5), "std": round(float(ts.std()), 5),
            "median": round(float(np.median(ts)), 5), "min": round(float(ts.min()), 5),
            "max": round(float(ts.max()), 5), "rsd": round(float(ts.std() / ts.mean()), 4)}


def measure_interp(reps=10):
    """The interpolation benchmark of Sec. 4.3 on the library's stand-alone
    interpolators: a natural cubic spline through y = x^2 on 512 random knots,
    and the 64 x 64 table of 128-knot splines with bilinear interpolation
    between rows for z = x^2 + y^2, each at 10^2 .. 10^8 random queries.
    Per size: the kernel alone (HIP events), and with the queries copied from
    pinned host memory and the results copied back, as the paper times its
    GPU routine; 10 repetitions each.  Mean relative residual against the
    analytic function at 10^6 queries."""
    import numpy as np
    import torch

    from paper_2510_02873_amd import _abi

    dev = torch.device("cuda", 0)
    g = torch.Generator(device=dev).manual_seed(4321)
    stream = torch.cuda.current_stream(dev)

    def knots(k, lo=0.0, hi=1.0):
        inner = torch.sort(torch.rand(k - 2, dtype=torch.float64, device=dev, generator=g) * (hi - lo) + lo)[0]
        return torch.cat([torch.tensor([lo], dtype=torch.float64, device=dev), inner,
                          torch.tensor([hi], dtype=torch.float64, device=dev)])

    x = knots(512)
    y = x * x
    M = torch.empty_like(x)
    _abi.pino_spline_build(x, y, M, torch.empty_like(x), stream=stream)
    xk, yk, dk = knots(64), knots(64), knots(128)
    F = (xk[:, None, None] ** 2 + yk[None, :, None] ** 2).expand(64, 64, 128).contiguous()
    tab = torch.empty(2 * F.numel(), dtype=torch.float64, device=dev)
    _abi.pino_table_build(dk, F, tab, torch.empty(F.numel(), dtype=torch.float64, device=dev), stream=stream)

    def timed(fn):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        fn()
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return [e0.elapsed_time(e1) for e0, e1 in ev]

    out = {"spline": [], "table": []}
    for e in range(2, 9):
        m = 10 ** e
        q = [torch.rand(m, dtype=torch.float64, device=dev, generator=g) for _ in range(3)]
        r = torch.empty(m, dtype=torch.float64, device=dev)
        hq = [t.cpu().pin_memory() for t in q]
        hr = torch.empty(m, dtype=torch.float64).pin_memory()

        def spline():
            _abi.pino_spline_eval(x, y, M, q[0], r, stream=stream)

        def spline_io():
            q[0].copy_(hq[0], non_blocking=True)
            spline()
            hr.copy_(r, non_blocking=True)

        def table():
            _abi.pino_table_eval(xk, yk, dk, tab, q[0], q[1], q[2], r, stream=stream)

        def table_io():
            for t, h in zip(q, hq):
                t.copy_(h, non_blocking=True)
            table()
            hr.copy_(r, non_blocking=True)

        for name, k, kio in (("spline", spline, spline_io), ("table", table, table_io)):
            tk, tio = timed(k), timed(kio)
            out[name].append({"queries": m, "kernel_ms": _stats_ms(tk), "with_transfers_ms": _stats_ms(tio)})
        if m == 10 ** 6:
            spline()
            exact = q[0] * q[0]
            out["spline_mean_rel_residual"] = float(((r - exact).abs() / exact).mean().item())
            table()
            exact = q[0] * q[0] + q[1] * q[1]
            out["table_mean_rel_residual"] = float(((r - exact).abs() / exact).mean().item())
        del q, r, hq, hr
        log(f"interpolation sweep: 10^{e} queries done")
    for name in ("spline", "table"):
        last = out[name][-1]
        out[name + "_queries_per_s_at_1e8"] = round(1e8 / (last["kernel_ms"]["median"] * 1e-3), 1)
    out["setup"] = ("natural spline y=x^2 on 512 random knots in [0,1]; 64x64 table of 128-knot splines, "
                    "z=x^2+y^2, random knots; uniform random queries; 10 repetitions per size")
    return out


def measure_field(P, col, dk, radii, n, n_side, cfg, stream, F64, R64, steps, col_tables):
    """The Hessian stage on the device feeding the collapse with no host
    round trip (pino_field_collapse): per radius, delta(k) -> six weighted
    copies -> six inverse real FFTs (hipFFT) -> the same FP64 collapse
    kernel.  Reports evaluations/s with the FFTs included, the Hessian stage
    alone, and the agreement with the plain run on the generator's Hessians."""
    import torch

    last = len(radii) - 1
    flags = P.PINO_EVAL_RESET | P.PINO_EVAL_FINALIZE
    with P.Field(n_side, cfg["box"]) as f:
        Ff, Rf, Af = col.outputs(n)
        items = [P.make_item(None, Ff, Rf, Af if r == last else None, radius_index=r, n=n)
                 for r in range(len(radii))]
        ms = _time_steps(lambda: f.collapse(col.ctx, dk, radii, items, flags=flags, stream=stream), steps, stream)
        H = torch.empty((6, n), dtype=torch.float64, device=dk.device)

        def hstep():
            for R in radii:
                f.hessian(dk, R, H, stream=stream)

        ms_h = _time_steps(hstep, steps, stream)
        del H
        # the same from a mixed-precision context: FP32 products and FP32
        # inverse transforms feed the mixed kernel
        mcol = P.Collapse(col_tables, precision=P.PINO_MIXED)
        Fm, Rm, Am = mcol.outputs(n)
        mitems = [P.make_item(None, Fm, Rm, Am if r == last else None, radius_index=r, n=n)
                  for r in range(len(radii))]
        ms_m = _time_steps(lambda: f.collapse(mcol.ctx, dk, radii, mitems, flags=flags, stream=stream), steps,
                           stream)
        mcol.close()
    big = F64 > 1e-6
    rel = ((1 / Ff[big] - 1 / F64[big]).abs() * F64[big]).max().item()
    res = {"value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s", "ms_per_step": round(ms, 4),
           "mixed_value": round(n * len(radii) / (ms_m * 1e-3), 1), "mixed_ms_per_step": round(ms_m, 4),
           "hessian_stage_ms_per_step": round(ms_h, 4),
           "workload": f"delta(k) of the same {n_side}^3 field -> {len(radii)} radii, FFTs included",
           "max_rel_Dc_vs_generator_hessians": rel,
           "index_mismatch_frac": float((Rf != R64).double().mean().item())}
    log(f"field-fed collapse {res['value']:.3e} evals/s ({ms:.2f} ms/step, Hessian stage {ms_h:.2f} ms); "
        f"mixed {res['mixed_value']:.3e}")
    return res


def measure_surrogate(P, slabs, radii, sig, n, a, D, cfg, n_side, stream, F64, R64, steps,
                      train_steps=TRAIN_STEPS, blob_path=None, blob_out=None, method=None):
    """Learned surrogate + certify on the same FP64 fields: train the network
    with the library's kernels on 20M (inputs, target) pairs from the
    benchmark fields and four perturbed cosmologies (untimed), then time the
    certified collapse.  Reports evals/s, the certified / full-solve / gated
    counts and the error against the plain FP64 run on the same Hessians
    (the certificate bounds it by certify_rtol).  blob_path: take the network
    from that file instead of training (profiling runs reuse the bench's
    network); blob_out: write the trained network there.  method: the
    collapse condition (PINO_CLASSIC by default; with PINO_CLASSIC_LCDM the
    targets, the certificate and the full solve are the LCDM ones, and F64,
    R64 the plain LCDM run)."""
    import numpy as np
    import torch

    import synth
    from paper_2510_02873_amd import _abi, surrogate

    method = P.PINO_CLASSIC if method is None else method
    if blob_path:
        blob = open(blob_path, "rb").read()
        return _time_surrogate(P, blob, slabs, radii, sig, n, a, D, cfg, stream, F64, R64, steps,
                               {"loaded_from": os.path.basename(blob_path)}, method)
    t0 = time.time()
    om = cfg["cosmo"].omega_m
    perturbed = [synth.Cosmology(0.27, 0.8), synth.Cosmology(0.33, 0.8), synth.Cosmology(0.30, 0.75),
                 synth.Cosmology(0.30, 0.85)]
    tables = [(a, D, om)] + [(*synth.growth_table(c.omega_m), c.omega_m) for c in perturbed]
    pick = list(range(0, len(radii), 6))
    n_slabs = len(pick) + 2 * len(perturbed)
    per = 20_000_000 // n_slabs + 1
    fields = [(slabs[r], sig[r], 0) for r in pick]
    x0, w0 = surrogate.training_pairs(fields, tables, per_slab=per, method=method)
    xs, ws = [x0], [w0]
    for k, c in enumerate(perturbed):
        fld = synth.fields.field(n_side, cfg["box"], 51 + k, c, device=slabs[0].device)
        sp = synth.grid_sigma_gauss(n_side, cfg["box"], [4.0, 1.0], c)
        pf = [(fld.hessian(R), sR, k + 1) for R, sR in zip([4.0, 1.0], sp)]
        x, w = surrogate.training_pairs(pf, tables, per_slab=per, method=method)
        xs.append(x)
        ws.append(w)
        del fld, pf
    x = torch.cat(xs)[:20_000_000].contiguous()
    w = torch.cat(ws)[:20_000_000].contiguous()
    del xs, ws, x0, w0
    n_pairs = x.shape[0]
    log(f"surrogate: {n_pairs} training pairs in {time.time() - t0:.1f}s")
    t1 = time.time()
    blob, _, hist = surrogate.train(x, w, steps=train_steps, batch=16384, lr_max=3e-3, seed=7, log_every=10000,
                                    bf16_forward=True,
                                    log=lambda m: log(m))
    train_s = time.time() - t1
    del x, w
    if blob_out:
        with open(blob_out, "wb") as f:
            f.write(blob)
    training = {"pairs": int(n_pairs), "steps": train_steps, "batch": 16384, "bf16_forward": True,
                "seconds": round(train_s, 1), "final_loss": hist[-1][1] if hist else None}
    return _time_surrogate(P, blob, slabs, radii, sig, n, a, D, cfg, stream, F64, R64, steps, training, method)


def _time_surrogate(P, blob, slabs, radii, sig, n, a, D, cfg, stream, F64, R64, steps, training, method):
    import numpy as np

    from paper_2510_02873_amd import _abi
    om = cfg["cosmo"].omega_m
    n_side = round(n ** (1.0 / 3.0))
    last = len(radii) - 1
    scol = P.Collapse([(a, D, om)], method=method, precision=P.PINO_SURROGATE, mlp_blob=blob)
    Fs, Rs, As = scol.outputs(n)
    items = [scol.item(slabs[r], Fs, Rs, As if r == last else None, radius_index=r, sigma_R=sig[r])
             for r in range(len(radii))]

    def sstep():
        for r, it in enumerate(items):
            scol.eval([it], reset=(r == 0), finalize=(r == last), stream=stream)

    sstep()
    _abi.pino_collapse_surrogate_stats(scol.ctx, reset=True)
    sstep()
    st = _abi.pino_collapse_surrogate_stats(scol.ctx, reset=True)
    ms = _time_steps(sstep, steps, stream)
    big = F64 > 1e-6
    rel = ((1 / Fs[big] - 1 / F64[big]).abs() * F64[big]).cpu().numpy()
    consulted = st["certified"] + st["fallback"]
    total = consulted + st["gated"]
    res = {"value": round(n * len(radii) / (ms * 1e-3), 1), "unit": "evals/s", "ms_per_step": round(ms, 4),
           "dtype": "bf16 MFMA network (fp32 accumulate), fp64 inputs, eigen and Newton certificate",
           "workload": f"same {n_side}^3 x {len(radii)} fp64 fields",
           "certified": st["certified"], "fallback": st["fallback"], "gated_solved": st["gated_solved"],
           "gated_zero": st["gated_zero"],
           "fallback_fraction_of_consulted": round(st["fallback"] / max(consulted, 1), 4),
           "full_solve_fraction_of_all": round(st["full_solve"] / max(total, 1), 4),
           "rel_Dc_vs_fp64_field": {"max": float(rel.max()), "p99.9": float(np.percentile(rel, 99.9)),
                                    "mean": float(rel.mean())},
           "index_mismatch_frac": float((Rs != R64).double().mean().item()),
           "training": training,
           "condition": "LCDM LPT coefficients" if method == P.PINO_CLASSIC_LCDM else "EdS LPT coefficients"}
    scol.close()
    log(f"surrogate+certify {res['value']:.3e} evals/s, fallback {res['fallback_fraction_of_consulted']:.3f} of "
        f"consulted, full solve {res['full_solve_fraction_of_all']:.3f} of all, max rel D_c vs fp64 "
        f"{res['rel_Dc_vs_fp64_field']['max']:.2e}")
    res["blob"] = blob
    return res


def _probes():
    import ctypes
    from paper_2510_02873_amd import build as libbuild
    L = ctypes.CDLL(libbuild.PROBES)
    L.pino_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    L.pino_probe_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_void_p]
    L.pino_probe_fma_f64.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    for f in (L.pino_probe_copy, L.pino_probe_stream, L.pino_probe_fma_f64):
        f.restype = ctypes.c_int
    return L


def measure_ceilings(slabs, n, stream, reps=10):
    """Ceilings measured on this GPU next to the spec sheet's: a streaming
    copy (2 GiB read + 2 GiB written), the headline kernel's own data
    movement with no arithmetic (six FP64 Hessian streams, Fmax and Rmax
    read and written back as whole lines: 72 B per particle, on the
    benchmark's resident fields), and independent FP64 FMA chains."""
    import ctypes
    import torch

    L = _probes()
    dev = slabs[0].device
    h = stream.cuda_stream

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    nbytes = 2 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ms = timed(lambda: L.pino_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes // 16, h))
    out["copy_GBps"] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del src, dst
    F = torch.zeros(n, dtype=torch.float64, device=dev)
    R = torch.full((n,), -1, dtype=torch.int32, device=dev)
    ptrs = (ctypes.c_void_p * 6)(*[slabs[0][c].data_ptr() for c in range(6)])
    ms = timed(lambda: L.pino_probe_stream(ptrs, F.data_ptr(), R.data_ptr(), n, 1, h))
    out["collapse_pattern_GBps"] = round(72 * n / (ms * 1e-3) / 1e9, 1)
    out["collapse_pattern_us_per_launch"] = round(ms * 1e3, 2)
    del F, R
    blocks, iters = 256 * 16, 4096
    buf = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    ms = timed(lambda: L.pino_probe_fma_f64(buf.data_ptr(), blocks, iters, h))
    out["fp64_fma_TFs"] = round(blocks * 256 * 8 * iters * 2 / (ms * 1e-3) / 1e12, 2)
    out["probes"] = ("copy: 16 B per lane, nontemporal loads; collapse pattern: six f64 SoA streams (nontemporal) "
                     "+ Fmax/Rmax read and written as whole lines, pairs of particles per lane; fma: 8 "
                     "independent f64 FMA chains per lane, 4096 blocks of 256")
    log(f"ceilings: copy {out['copy_GBps']} GB/s, collapse pattern {out['collapse_pattern_GBps']} GB/s "
        f"({out['collapse_pattern_us_per_launch']} us), FP64 FMA {out['fp64_fma_TFs']} TF/s")
    return out


def measure_512(P, blob, steps=1):
    """The 512^3 x 40-radius configuration (one GPU's share of a 2048^3 run,
    seed 3, a field the surrogate never saw in training): per radius the
    FP64 Hessians come from the device's Hessian stage (pino_field) and the
    FP32 slab is their rounded copy; the mixed-precision path (FP32 slab)
    and the surrogate + certify path (FP64 Hessians) are each timed per
    launch with HIP events on the launch stream, the Hessian stage excluded.
    Errors of both against the FP64 oracle on a seeded sample of 20k
    particles over all 40 radii."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2510_02873_amd import _abi

    cfg = synth.config("C3")
    n_side, box, radii, cosmo = cfg["n_side"], cfg["box"], cfg["radii"], cfg["cosmo"]
    n = n_side ** 3
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    a, D = synth.growth_table(cosmo.omega_m, cfg["n_growth"])
    sig = synth.grid_sigma_gauss(n_side, box, radii, cosmo)
    t0 = time.time()
    fld = synth.fields.field(n_side, box, cfg["seed"], cosmo, device=dev)
    dk = fld.dk.contiguous()
    del fld
    torch.cuda.empty_cache()
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(n, size=20000, replace=False))
    tidx = torch.from_numpy(idx).to(dev)
    H64 = torch.empty((6, n), dtype=torch.float64, device=dev)
    H32 = torch.empty((6, n), dtype=torch.float32, device=dev)
    mix = P.Collapse([(a, D, cosmo.omega_m)], precision=P.PINO_MIXED)
    sur = P.Collapse([(a, D, cosmo.omega_m)], precision=P.PINO_SURROGATE, mlp_blob=blob)
    Fm, Rm, Am = mix.outputs(n)
    Fs, Rs, As = sur.outputs(n)
    last = len(radii) - 1
    t_mix, t_sur = [], []
    sample = []
    _abi.pino_collapse_surrogate_stats(sur.ctx, reset=True)
    with P.Field(n_side, box) as f:
        for step in range(steps):
            for r, R in enumerate(radii):
                f.hessian(dk, R, H64, stream=stream)
                H32.copy_(H64)
                if step == 0:
                    sample.append(H64[:, tidx].cpu().numpy())
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                ev[0].record(stream)
                mix.apply(H32, r, Fm, Rm, Am if r == last else None, reset=(r == 0), finalize=(r == last),
                          stream=stream)
                ev[1].record(stream)
                ev[2].record(stream)
                sur.apply(H64, r, Fs, Rs, As if r == last else None, reset=(r == 0), finalize=(r == last),
                          sigma_R=sig[r], stream=stream)
                ev[3].record(stream)
                torch.cuda.synchronize()
                t_mix.append(ev[0].elapsed_time(ev[1]))
                t_sur.append(ev[2].elapsed_time(ev[3]))
            log(f"512^3 x {len(radii)}: pass {step + 1}/{steps} done ({time.time() - t0:.0f}s)")
    st = _abi.pino_collapse_surrogate_stats(sur.ctx)
    got_m = [t[tidx].cpu().numpy() for t in (Fm, Rm, Am)]
    got_s = [t[tidx].cpu().numpy() for t in (Fs, Rs, As)]
    mix.close()
    sur.close()
    del H32, Fs, Rs, As
    torch.cuda.empty_cache()
    try:
        resident = _c3_resident(P, dk, H64, n_side, box, radii, a, D, cosmo, tidx, (Fm, Rm, Am), stream)
    except (RuntimeError, torch.cuda.OutOfMemoryError) as e:
        resident = {"error": str(e)[:300]}
        log(f"512^3 resident leg failed: {e}")
    del H64, dk, Fm, Rm, Am
    torch.cuda.empty_cache()
    ref = oracle.collapse(sample, oracle.Growth(a, D))

    def errs(got):
        Fr, Rr, Ar = ref
        big = Fr >= 1e-6
        both = big & (got[0] > 0)
        rD = np.abs(1 / got[0][both] - 1 / Fr[both]) * Fr[both]
        fin = np.isfinite(Ar) & np.isfinite(got[2])
        ra = np.abs(got[2][fin] - Ar[fin]) / Ar[fin]
        stat = lambda x: {"max": float(x.max()), "p99.9": float(np.percentile(x, 99.9)), "mean": float(x.mean())}
        return {"rel_Dc": stat(rD), "rel_acoll": stat(ra), "index_mismatches": int(np.sum(got[1] != Rr)),
                "collapse_set_differs": int(np.sum((got[0] > 0) != (Fr > 0))), "sample": int(Fr.size)}

    evals = n * len(radii) * steps
    wl = f"512cube-{len(radii)}radii"
    out = {"mixed": {"workload": wl, "value": round(evals / (sum(t_mix) * 1e-3), 1), "unit": "evals/s",
                     "ms_per_pass": round(sum(t_mix) / steps, 3),
                     "dtype": "f32 slab (rounded fp64 field), f32 eigen/interp, f64 root",
                     "vs_fp64_oracle_on_fp64_field": errs(got_m),
                     "roofline": step_roofline(n * len(radii) * (24 + 8) + n * 20, sum(t_mix) / steps)},
           "surrogate": {"workload": wl, "value": round(evals / (sum(t_sur) * 1e-3), 1), "unit": "evals/s",
                         "ms_per_pass": round(sum(t_sur) / steps, 3),
                         "dtype": "fp64 inputs/eigen/certificate, bf16 MFMA network",
                         "held_out": "field seed 3 (training used the 256^3 seed-2 fields and seeds 51-54)",
                         "certified": st["certified"], "fallback": st["fallback"],
                         "gated_solved": st["gated_solved"], "gated_zero": st["gated_zero"],
                         "fallback_fraction_of_consulted": round(st["fallback"] / max(1, st["certified"] +
                                                                                     st["fallback"]), 4),
                         "full_solve_fraction_of_all": round(st["full_solve"] / max(1, evals), 4),
                         "vs_fp64_oracle_on_fp64_field": errs(got_s)},
           "timing": "sum of per-launch HIP-event times over the radii (Hessian stage excluded)"}
    got_r = resident.pop("_got", None)
    if got_r is not None:
        resident["vs_fp64_oracle_on_fp64_field"] = errs(got_r)
        resident["workload"] = wl
    out["mixed_resident"] = resident
    log(f"512^3: mixed {out['mixed']['value']:.3e} evals/s (all radii resident: "
        f"{resident.get('value', float('nan')):.3e}), surrogate {out['surrogate']['value']:.3e} evals/s; "
        f"surrogate max rel D_c vs fp64 {out['surrogate']['vs_fp64_oracle_on_fp64_field']['rel_Dc']['max']:.2e}")
    return out


def _c3_resident(P, dk, H64, n_side, box, radii, a, D, cosmo, tidx, per_radius, stream, passes=3):
    """The 512^3 x 40-radius mixed-precision workload with every FP32 radius
    resident (129 GB, from the same Hessian stage as the per-radius leg): one
    persistent batched launch per pass, replayed from a HIP graph, tiles and
    grid autotuned on the data; the running maxima stay in registers across
    the radii, so a pass reads 24 B per evaluation plus 20 B per particle.
    Its outputs are checked to equal the per-radius evals' bit for bit."""
    import torch

    from paper_2510_02873_amd import _abi

    n = n_side ** 3
    t0 = time.time()
    slabs = []
    with P.Field(n_side, box) as f:
        for radius in radii:
            f.hessian(dk, radius, H64, stream=stream)
            s = torch.empty((6, n), dtype=torch.float32, device=H64.device)
            s.copy_(H64)
            slabs.append(s)
    torch.cuda.synchronize()
    log(f"512^3: {len(radii)} FP32 radii resident in {time.time() - t0:.1f}s")
    col = P.Collapse([(a, D, cosmo.omega_m)], precision=P.PINO_MIXED)
    F, R, A = col.outputs(n)
    b = _abi.Batch(col.ctx, [{"h": slabs, "Fmax": F, "Rmax": R, "a_coll": A, "cosmo": 0}],
                   flags=P.PINO_EVAL_RESET | P.PINO_EVAL_FINALIZE, autotune=True)
    conf = b.config()
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        ms = _time_steps(lambda: b.graph_launch(gs), passes, gs)
    Fp, Rp, Ap = per_radius
    same = bool(torch.equal(F, Fp) and torch.equal(R, Rp) and torch.equal(A, Ap))
    got = [t[tidx].cpu().numpy() for t in (F, R, A)]
    b.close()
    col.close()
    del slabs, F, R, A
    torch.cuda.empty_cache()
    evals = n * len(radii)
    return {"value": round(evals / (ms * 1e-3), 1), "unit": "evals/s", "ms_per_pass": round(ms, 3),
            "dtype": "f32 slab (rounded fp64 field), f32 eigen/interp, f64 root",
            "launch": "one persistent kernel per pass, HIP graph replay, all radii resident", "autotuned": conf,
            "identical_to_per_radius": same, "roofline": step_roofline(evals * 24 + n * 20, ms), "_got": got}


def measure_batched(P, steps):
    """C4: 64 realisations (grid sides uniform in 64..192, cell 0.78125 Mpc/h),
    each with its own cosmology and 512-point growth table, 20 radii 16 -> 1
    Mpc/h, FP64, every radius resident (182 GB).  One persistent launch per
    step, captured in a HIP graph, tiles and grid autotuned on the data."""
    import numpy as np
    import torch

    import synth
    from paper_2510_02873_amd import _abi

    cfg = synth.config("C4")
    reals = cfg["realisations"]
    radii = cfg["radii"]
    t0 = time.time()
    tables = [(*synth.growth_table(r["cosmo"].omega_m), r["cosmo"].omega_m) for r in reals]
    col = P.Collapse(tables, precision=P.PINO_FP64)
    descs, n_tot = [], 0
    for k, r in enumerate(reals):
        fld = synth.fields.field(r["n_side"], r["box"], r["seed"], r["cosmo"], device="cuda")
        n = r["n_side"] ** 3
        # component rows padded to an even length: every row starts 16-byte
        # aligned, which the two-particles-per-lane path needs
        slabs = [fld.hessian(R, out=torch.empty((6, n + (n & 1)), dtype=torch.float64, device="cuda")[:, :n])
                 for R in radii]
        del fld
        F, Rm, A = col.outputs(n)
        descs.append({"h": slabs, "Fmax": F, "Rmax": Rm, "a_coll": A, "cosmo": k})
        n_tot += n
        if k % 8 == 7:
            log(f"batched: {k + 1}/{len(reals)} realisations generated ({time.time() - t0:.0f}s)")
    torch.cuda.synchronize()
    log(f"batched: {len(reals)} realisations, {n_tot} particles x {len(radii)} radii generated in "
        f"{time.time() - t0:.1f}s")
    b = _abi.Batch(col.ctx, descs, flags=P.PINO_EVAL_RESET | P.PINO_EVAL_FINALIZE, autotune=True)
    conf = b.config()
    gstream = torch.cuda.Stream()          # graphs are captured on a non-null stream
    with torch.cuda.stream(gstream):
        ms = _time_steps(lambda: b.graph_launch(gstream), steps, gstream)
    evals = n_tot * len(radii)
    bytes_launch = n_tot * (48 * len(radii) + 20)
    res = {"value": round(evals / (ms * 1e-3), 1), "unit": "evals/s", "ms_per_step": round(ms, 4),
           "workload": f"{len(reals)} realisations, sides 64..192, {n_tot} particles x {len(radii)} radii, "
                       "own cosmology each, fp64, all radii resident",
           "launch": "one persistent kernel per step, HIP graph replay", "autotuned": conf,
           "roofline": {"bound": "hbm", "achieved": round(bytes_launch / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(bytes_launch / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "bytes_per_launch": int(bytes_launch)}}
    # spot parity: a few particles of a few realisations against the oracle
    import oracle
    rng = np.random.default_rng(77)
    worst = 0.0
    for k in rng.choice(len(reals), size=3, replace=False):
        d = descs[k]
        n = d["Fmax"].numel()
        idx = torch.from_numpy(np.sort(rng.choice(n, size=min(4096, n), replace=False))).cuda()
        ref = oracle.collapse([h[:, idx].cpu().numpy() for h in d["h"]], oracle.Growth(*tables[k][:2]))
        F = d["Fmax"][idx].cpu().numpy()
        big = ref[0] >= 1e-6
        worst = max(worst, float(np.max(np.abs(1 / F[big] - 1 / ref[0][big]) * ref[0][big])))
    res["parity_sample_max_rel_Dc"] = worst
    b.close()
    col.close()
    del descs
    torch.cuda.empty_cache()
    log(f"batched {res['value']:.3e} evals/s ({conf})")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24,
                    help="particles in the oracle sample (2^24: every particle of the 256^3 field, ~15 s of oracle time)")
    ap.add_argument("--n-side", type=int, default=None, help="override the grid side (testing only)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (mixed precision, Tabulated) on the same fields")
    ap.add_argument("--save-blob", default=None, help="write the trained surrogate network to this file")
    ap.add_argument("--load-blob", default=None,
                    help="take the surrogate network from this file instead of training one (profiling runs)")
    ap.add_argument("--no-512", action="store_true",
                    help="skip the 512^3 x 40-radius mixed-precision and surrogate legs")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched 64-realisation workload (182 GB of resident Hessians)")
    ap.add_argument("--train-steps", type=int, default=TRAIN_STEPS,
                    help="optimiser steps of the surrogate's (untimed) training; counter-collection runs, which "
                         "serialise every dispatch, shorten it")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB device-to-device once, so HBM "
                         "counters can be scaled against a transfer of known size")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1 (the per-particle "
                                   "collapse path has no cross-GPU step, see the design notes on sharding)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_02873_amd as P
    import synth

    if not os.path.exists(P.LIB_PATH):
        from paper_2510_02873_amd import build as libbuild
        libbuild.build()

    cfg = synth.config("C2")
    n_side = args.n_side or cfg["n_side"]
    radii = cfg["radii"]
    n = n_side ** 3
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    t0 = time.time()
    a, D = synth.growth_table(cfg["cosmo"].omega_m, cfg["n_growth"])
    fld = synth.fields.field(n_side, cfg["box"], cfg["seed"], cfg["cosmo"], device=dev)
    slabs = [fld.hessian(R) for R in radii]
    dk = fld.dk.contiguous()      # delta(k), for the device Hessian stage leg
    del fld
    torch.cuda.synchronize()
    log(f"inputs ready: n={n} radii={len(radii)} in {time.time() - t0:.1f}s "
        f"({len(radii) * 48 * n / 1e9:.1f} GB of Hessians resident)")

    if args.calib_copy_mib > 0:
        src = torch.empty(args.calib_copy_mib << 17, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst

    col = P.Collapse([(a, D)], device=0)
    Fmax, Rmax, ac = col.outputs(n)
    stream = torch.cuda.current_stream(dev)

    last = len(radii) - 1
    # a_coll is produced once, from the running maximum, on the last radius
    # (PINO_EVAL_FINALIZE; identical to updating it at every radius)
    items = [col.item(slabs[r], Fmax, Rmax, ac if r == last else None, radius_index=r)
             for r in range(len(radii))]

    # untimed pass: how many particles update their max at each radius
    updates = []
    prev = None
    for r in range(len(radii)):
        col.eval([items[r]], reset=(r == 0), finalize=(r == last), stream=stream)
        cur = Fmax.clone()
        updates.append(int(n if prev is None else (cur != prev).sum().item()))
        prev = cur
    del prev, cur
    bytes_per_launch = [algorithmic_bytes(n, u, r == 0, r == last) for r, u in enumerate(updates)]

    def step(events=None):
        for r, it in enumerate(items):
            if events is not None:
                events[r][0].record(stream)
            col.eval([it], reset=(r == 0), finalize=(r == last), stream=stream)
            if events is not None:
                events[r][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(args.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    log(f"timed {args.steps} steps: {total_ms:.2f} ms (wall {wall * 1e3:.2f} ms)")

    # the spread of single launches, from as many steps again after the
    # timed region with an event pair around every launch (those events put
    # a few microseconds between launches, about 3 % of a step, so they stay
    # out of the timed region)
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in radii]
          for _ in range(args.steps)]
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    launch_ms = np.array([[e[0].elapsed_time(e[1]) for e in ev[k]] for k in range(args.steps)])

    evals_per_step = n * len(radii)
    ms_per_step = total_ms / args.steps
    value = evals_per_step / (ms_per_step * 1e-3)

    # roofline of the collapse kernel: algorithmic bytes of each launch over
    # its mean duration in the timed region (a step is the 25 launches of
    # this kernel back to back, so the timed region over the launch count is
    # that mean, gaps between launches included)
    mean_launch_ms = total_ms / (args.steps * len(radii))
    mean_bytes = float(np.mean(bytes_per_launch))
    achieved_gbs = mean_bytes / (mean_launch_ms * 1e-3) / 1e9
    # measured HBM traffic and FP64 FLOPs per launch (scaled rocprofv3
    # counters), valid only while the loaded kernel's machine code is the one
    # that was profiled
    from paper_2510_02873_amd.profiling import kernel_digest, read_profile
    prof = read_profile(PROFILE)
    valid = prof.get("kernel_digest") == kernel_digest("k_classic_f64", P._abi.LIB_PATH)
    traffic = prof.get("traffic_bytes_per_launch") if valid else None
    flops = prof.get("fp64_flops_per_launch") if valid else None
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / 1e9, 4),
                "traffic_unit": "GB per launch",
                "kernel": "k_classic_f64", "mean_launch_us": round(mean_launch_ms * 1e3, 2),
                "mean_launch_from": "timed region (HIP events on the kernel's stream) / launches",
                "per_launch_events": {"mean_us": round(float(launch_ms.mean()) * 1e3, 2),
                                      "median_us": round(float(np.median(launch_ms)) * 1e3, 2),
                                      "min_us": round(float(launch_ms.min()) * 1e3, 2),
                                      "rsd": round(float(launch_ms.std() / launch_ms.mean()), 4)},
                "bytes_per_launch": int(mean_bytes), "update_fraction": round(
                    float(np.mean([u / n for u in updates[1:]])), 4)}
    if traffic is not None:
        roofline["traffic_GBps"] = round(traffic / (mean_launch_ms * 1e-3) / 1e9, 1)
    # FP64 roofline of the same kernel: counter FLOPs per launch over the live
    # mean launch duration, against the FP64 vector peak
    roofline["fp64"] = None if flops is None else {
        "achieved": round(flops / (mean_launch_ms * 1e-3) / 1e12, 3), "peak": FP64_PEAK_TFS,
        "unit": "TFLOP/s", "frac": round(flops / (mean_launch_ms * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
        "flops_per_eval": round(flops / n, 1)}

    extras = {}
    blob = None
    try:
        roofline["measured_ceilings"] = measure_ceilings(slabs, n, stream)
        mc = roofline["measured_ceilings"]
        roofline["frac_of_measured_copy"] = round(achieved_gbs / mc["copy_GBps"], 4)
        roofline["launch_vs_collapse_pattern"] = round(mc["collapse_pattern_us_per_launch"] /
                                                       (mean_launch_ms * 1e3), 4)
        if roofline.get("fp64"):
            roofline["fp64"]["frac_of_measured_fma"] = round(roofline["fp64"]["achieved"] / mc["fp64_fma_TFs"], 4)
    except (OSError, RuntimeError) as e:
        roofline["measured_ceilings"] = {"error": str(e)[:200]}
    if not args.no_extras:
        extras = measure_extras(P, col, slabs, radii, n, a, D, cfg, n_side, stream, Fmax, Rmax, ac, args.steps, dk,
                                updates, args.train_steps, plain_ms=ms_per_step, blob_path=args.load_blob,
                                blob_out=args.save_blob)
        blob = extras.pop("_blob", None)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(12345)
        m = min(args.cpu_sample, n)
        idx = torch.from_numpy(np.sort(rng.choice(n, size=m, replace=False))).to(dev)
        g = oracle.Growth(a, D)
        log(f"cpu baseline: oracle on {m} particles x {len(radii)} radii, {oracle.threads()} threads")
        rF, rR, rA = np.zeros(m), np.full(m, -1, np.int32), np.full(m, np.inf)
        dt = 0.0
        for r in range(len(radii)):
            sample = slabs[r][:, idx].cpu().numpy()       # gathered outside the timed call
            c0 = time.perf_counter()
            oracle.update_radius(sample, r, g, rF, rR, rA, reset=(r == 0))
            dt += time.perf_counter() - c0
        cpu = {"value": round(m * len(radii) / dt, 1), "unit": "evals/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"{m} seeded-random particles of the same {n_side}^3 fields x all {len(radii)} radii "
                         f"({dt:.1f} s of oracle time)"}
        # single-core rate on the first 2^16 sampled particles, all radii
        m1 = min(m, 1 << 16)
        nthreads = oracle.threads()
        oracle.set_threads(1)
        z = (np.zeros(m1), np.full(m1, -1, np.int32), np.full(m1, np.inf))
        dt1 = 0.0
        for r in range(len(radii)):
            sample = slabs[r][:, idx[:m1]].cpu().numpy()
            c0 = time.perf_counter()
            oracle.update_radius(sample, r, g, *z, reset=(r == 0))
            dt1 += time.perf_counter() - c0
        oracle.set_threads(nthreads)
        cpu["value_1core"] = round(m1 * len(radii) / dt1, 1)
        # the sampled particles also serve as a parity spot check of this run
        got_F = Fmax[idx].cpu().numpy()
        got_R = Rmax[idx].cpu().numpy()
        got_a = ac[idx].cpu().numpy()
        big = rF >= 1e-6
        rel = float(np.max(np.abs(1 / got_F[big] - 1 / rF[big]) * rF[big])) if big.any() else 0.0
        fin = np.isfinite(rA)
        rel_a = float(np.max(np.abs(got_a[fin] - rA[fin]) / rA[fin])) if fin.any() else 0.0
        cpu["parity_max_rel_Dc"] = rel
        cpu["parity_max_rel_acoll"] = rel_a
        cpu["parity_index_mismatches"] = int(np.sum(got_R != rR))
        log(f"cpu baseline {cpu['value']:.3e} evals/s; sample parity max rel D_c {rel:.2e} a_coll {rel_a:.2e}")

    run_512 = blob is not None and not args.no_512 and args.n_side is None
    run_batched = not args.no_batched and args.n_side is None
    if run_512 or run_batched:
        del slabs, items
        torch.cuda.empty_cache()
    if run_512:
        try:
            extras["c512"] = measure_512(P, blob)
        except (RuntimeError, torch.cuda.OutOfMemoryError) as e:
            extras["c512"] = {"error": str(e)[:300]}
            log(f"512^3 leg failed: {e}")
        torch.cuda.empty_cache()
    if run_batched:
        try:
            extras["batched"] = measure_batched(P, max(3, args.steps // 2))
        except (RuntimeError, torch.cuda.OutOfMemoryError) as e:
            extras["batched"] = {"error": str(e)[:300]}
            log(f"batched leg failed: {e}")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded Gaussian BBKS field, FFT Hessians (no dataset)",
        "config": {"workload": f"plain-fp64-classic-{n_side}cube-{len(radii)}radii",
                   "particles": n, "radii": len(radii), "evals_per_step": evals_per_step,
                   "box_mpc_h": cfg["box"], "growth_knots": cfg["n_growth"], "method": "classic",
                   "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    col.close()


if __name__ == "__main__":
    main()
