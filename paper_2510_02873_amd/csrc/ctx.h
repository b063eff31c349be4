// Library context behind the opaque pino_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

// Orders the calls of one handle that share its device scratch (a per-radius
// table, a queue, FFT work buffers) when the caller moves between streams:
// after each call an event is recorded on the call's stream, and a call on a
// different stream first waits for it.  Work the caller captures into a graph
// is not ordered this way (no event is recorded or waited on a capturing
// stream); ordering such graphs against other streams is the caller's.
struct StreamOrder {
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    bool capturing = false;

    hipError_t create()
    {
        return hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    }
    void destroy()
    {
        if (ev)
            (void)hipEventDestroy(ev);
        ev = nullptr;
    }
    // before the call's first launch on s
    hipError_t enter(hipStream_t s)
    {
        if (!ev)
            return hipSuccess;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess)
            return e;
        capturing = cs != hipStreamCaptureStatusNone;
        if (!capturing && used && s != last)
            e = hipStreamWaitEvent(s, ev, 0);
        return e;
    }
    // after the call's last launch on s
    hipError_t leave(hipStream_t s)
    {
        if (!ev || capturing)
            return hipSuccess;
        last = s;
        used = true;
        return hipEventRecord(ev, s);
    }
};

struct pino_ctx {
    int device = 0;
    int method = 0;
    int precision = 0;
    int n_cosmo = 0;
    int cu_count = 1;
    int blocks_per_cu = 8;

    // growth tables [D | a | M] per cosmology, stride 3 * nk_max doubles
    int nk_max = 0;
    std::vector<int> nk;
    double* d_growth = nullptr;
    float* d_growth32 = nullptr;  // FP32 copy for the mixed-precision path

    // per cosmology interval index of the growth knots: [idx | need], stride
    // 2 * nb_max ints; bin geometry and whether the two-compare bound holds
    int nb_max = 0;
    int* d_gidx = nullptr;
    std::vector<int> nb;
    std::vector<float> gL0, gS;
    std::vector<int> gok;

    // tabulated method: dimensionless knots [x | y | delta], the interleaved
    // (F, M) table of the current radius
    int nx = 0, ny = 0, nd = 0;
    double* d_tknots = nullptr;
    // interval index of the table knots (x | y | delta bins), when it holds
    int* d_tidx = nullptr;
    int tindexed = 0;
    int tnb[3] = {0, 0, 0};
    double tk0[3] = {0.0, 0.0, 0.0};
    double tbpu[3] = {0.0, 0.0, 0.0};
    double* d_tab = nullptr;
    // natural-spline elimination coefficients of the dimensionless delta knots
    double* d_tcoef = nullptr;
    // mixed precision: FP32 knot-pair table (F_j, M_j, F_j+1, M_j+1) per row
    void* d_tab32 = nullptr;
    // homogeneous-ellipsoid table fill: the growing mode's D(a = 1) of each
    // cosmology in that integration's normalisation (computed at first use)
    std::vector<double> ell_D1;

    // spline-build scratch
    double* d_tmp = nullptr;

    // PINO_CLASSIC_LCDM: per cosmology [k2 | k3a | k3b | m2 | m3a | m3b] at
    // the growth knots (stride 6 * nk_max): the LCDM growth ratios of the
    // LPT terms and their natural-spline second derivatives in D
    double* d_kap = nullptr;
    // the same splines as power-form coefficients per interval
    // (kappa_poly_doubles(nk_max) per cosmology), when they fit in LDS
    double* d_kpoly = nullptr;
    bool lcdm_poly = false;
    // per cosmology, bounds on |d k / d ln D| of the three ratio splines over
    // the whole table (the surrogate's LCDM certificate)
    std::vector<double> kslope;
    // launch shape of the LCDM kernel: its LDS (knots, index and ratio splines)
    // limits the resident blocks per CU, so the grid is capped at what fits
    int lcdm_block = 512;
    int lcdm_resident = 1;

    // surrogate network: BF16 weight fragments, certificate tolerance,
    // counters (certified, fallback, gated), Omega_m per cosmology
    void* d_mlp = nullptr;
    double certify_rtol = 5e-7;
    int64_t* d_counters = nullptr;
    // surrogate: queue of deferred particle indices (chunk-relative), one
    // segment per block
    int32_t* d_queue = nullptr;
    int64_t queue_cap = 0;
    std::vector<double> omega;

    // orders evals across streams (contexts with per-context scratch: the
    // Tabulated table, the surrogate's queue and counters)
    StreamOrder order;

    bool broken = false;
    std::string err = "no error";
};
