// Host side of the C ABI declared in include/pino_collapse.h: argument
// validation, context lifetime, device tables and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pino_collapse.h"
#include "ctx.h"
#include "kernels_ellipsoid.h"
#include "kernels_fp64.h"
#include "kernels_lcdm.h"
#include "launch_ext.h"
#include "mlp_api.h"

using namespace pino;

namespace {

thread_local std::string g_init_error = "no error";

constexpr int kMaxGrowthKnots = 2048;
constexpr int64_t kMaxTableCells = int64_t(1) << 24;

bool strictly_increasing(const double* v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i]))
            return false;
    for (int i = 0; i + 1 < n; ++i)
        if (!(v[i + 1] > v[i]))
            return false;
    return true;
}

// Pure host checks of a configuration; no HIP call.
bool validate_config(const pino_config* cfg, std::string& why)
{
    if (!cfg) {
        why = "config is NULL";
        return false;
    }
    if (cfg->abi_version != PINO_ABI_VERSION) {
        why = "abi_version " + std::to_string(cfg->abi_version) + " != " + std::to_string(PINO_ABI_VERSION);
        return false;
    }
    if (cfg->method != PINO_CLASSIC && cfg->method != PINO_TABULATED && cfg->method != PINO_CLASSIC_LCDM) {
        why = "unknown method";
        return false;
    }
    if (cfg->precision != PINO_FP64 && cfg->precision != PINO_MIXED && cfg->precision != PINO_SURROGATE) {
        why = "unknown precision";
        return false;
    }
    if (cfg->device < 0) {
        why = "device < 0";
        return false;
    }
    if (cfg->n_cosmo < 1 || !cfg->growth) {
        why = "need at least one growth table";
        return false;
    }
    for (int c = 0; c < cfg->n_cosmo; ++c) {
        const pino_growth& g = cfg->growth[c];
        if (g.n < 4 || g.n > kMaxGrowthKnots || !g.a || !g.D) {
            why = "growth table " + std::to_string(c) + ": need 4 <= n <= 2048 and non-NULL a, D";
            return false;
        }
        if (!std::isfinite(g.omega_m)) {
            why = "growth table " + std::to_string(c) + ": omega_m must be finite";
            return false;
        }
        if (cfg->method == PINO_CLASSIC_LCDM && !(g.omega_m > 0.0 && g.omega_m <= 1.0)) {
            why = "growth table " + std::to_string(c) + ": the LCDM method needs 0 < omega_m <= 1";
            return false;
        }
        if (!strictly_increasing(g.a, g.n) || !strictly_increasing(g.D, g.n)) {
            why = "growth table " + std::to_string(c) + ": a and D must be finite and strictly increasing";
            return false;
        }
    }
    if (cfg->certify_rtol < 0.0 || !(cfg->certify_rtol < 1e-2)) {
        why = "certify_rtol must be in [0, 1e-2)";
        return false;
    }
    if (cfg->method == PINO_TABULATED) {
        const pino_table_knots* t = cfg->table;
        if (!t || !t->x || !t->y || !t->delta || t->nx < 2 || t->ny < 2 || t->nd < 4) {
            why = "tabulated method needs table knots with nx, ny >= 2 and nd >= 4";
            return false;
        }
        if ((int64_t)t->nx * t->ny * t->nd > kMaxTableCells) {
            why = "table larger than 2^24 cells";
            return false;
        }
        if (!strictly_increasing(t->x, t->nx) || !strictly_increasing(t->y, t->ny) ||
            !strictly_increasing(t->delta, t->nd)) {
            why = "table knots must be finite and strictly increasing";
            return false;
        }
        if (cfg->precision == PINO_SURROGATE) {
            why = "the surrogate replaces the Classic solve only";
            return false;
        }
    }
    if (cfg->precision == PINO_SURROGATE) {
        std::string mwhy;
        if (!mlp_blob_valid(cfg->mlp, cfg->mlp_bytes, mwhy)) {
            why = "surrogate weights: " + mwhy;
            return false;
        }
    }
    return true;
}

bool validate_items(const pino_ctx* ctx, const pino_item* items, int32_t n_items, uint32_t flags, std::string& why)
{
    if (n_items < 0) {
        why = "n_items < 0";
        return false;
    }
    if (n_items > 0 && !items) {
        why = "items is NULL";
        return false;
    }
    for (int32_t k = 0; k < n_items; ++k) {
        const pino_item& it = items[k];
        const std::string at = "item " + std::to_string(k) + ": ";
        if (it.n < 0) {
            why = at + "n < 0";
            return false;
        }
        if (it.cosmo < 0 || it.cosmo >= ctx->n_cosmo) {
            why = at + "cosmo index out of range";
            return false;
        }
        if (it.radius_index < 0) {
            why = at + "radius_index < 0";
            return false;
        }
        if (it.n == 0)
            continue;
        for (int c = 0; c < 6; ++c)
            if (!it.h[c]) {
                why = at + "Hessian component pointer is NULL";
                return false;
            }
        if (!it.Fmax || !it.Rmax) {
            why = at + "Fmax and Rmax must be non-NULL";
            return false;
        }
        if ((flags & PINO_EVAL_FINALIZE) && !it.a_coll) {
            why = at + "PINO_EVAL_FINALIZE needs a_coll";
            return false;
        }
        if ((ctx->method == PINO_TABULATED || ctx->precision == PINO_SURROGATE) &&
            !(std::isfinite(it.sigma_R) && it.sigma_R > 0.0)) {
            why = at + "sigma_R must be finite and > 0";
            return false;
        }
        if (ctx->method == PINO_TABULATED && !it.table_F) {
            why = at + "table_F is NULL";
            return false;
        }
    }
    return true;
}

pino_status hip_fail(pino_ctx* ctx, hipError_t e, const char* what)
{
    ctx->broken = true;
    ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return PINO_ERR_HIP;
}

#define PINO_HIP(ctx, call)                          \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess)                        \
            return hip_fail((ctx), e_, #call);       \
    } while (0)

// LDS per workgroup: growth knots + index bins, plus the table knots of the
// Tabulated method; kept within 64 KiB.  The surrogate kernel also holds the
// network's weight fragments and may use up to the 160 KiB a CDNA4
// workgroup can address (its limit is raised at init).
constexpr size_t kLdsBudget = 65536;
constexpr size_t kLdsMax = 163840;

int index_bins(int nk)
{
    return (int)std::min<int64_t>(4 * (int64_t)nk, (57344 - 24 * (int64_t)nk) / 4);
}

bool lds_fits(const pino_config* cfg, std::string& why)
{
    int nk_max = 0;
    for (int k = 0; k < cfg->n_cosmo; ++k)
        nk_max = std::max(nk_max, (int)cfg->growth[k].n);
    if (cfg->method == PINO_CLASSIC_LCDM) {
        const size_t need = cfg->precision == PINO_SURROGATE
                                ? surrogate_lds_bytes(nk_max, index_bins(nk_max), true)
                                : lcdm_lds_bytes(nk_max, index_bins(nk_max));
        if (need > kLdsMax) {
            why = "growth knots and LCDM coefficients need " + std::to_string(need) + " bytes of LDS, more than 160 KiB";
            return false;
        }
        return true;
    }
    if (cfg->precision == PINO_SURROGATE) {
        const size_t need = surrogate_lds_bytes(nk_max, index_bins(nk_max));
        if (need > kLdsMax) {
            why = "growth knots and network weights need " + std::to_string(need) + " bytes of LDS, more than 160 KiB";
            return false;
        }
        return true;
    }
    size_t need = growth_lds_bytes(nk_max, index_bins(nk_max));
    if (cfg->method == PINO_TABULATED)
        need += sizeof(double) * ((size_t)cfg->table->nx + cfg->table->ny + cfg->table->nd);
    if (need > kLdsBudget) {
        why = "growth and table knots need " + std::to_string(need) + " bytes of LDS, more than 64 KiB";
        return false;
    }
    return true;
}

// Interval index of one axis of dimensionless table knots k[n] (TabArgs):
// 4 (n - 1) uniform bins, each holding the interval at its low end less a
// margin of 1 % of a bin; false if more than kIndexCompares knots can follow
// inside a bin (the kernels then use the binary search) or if the margin is
// not far above the rounding of the bin arithmetic.
bool table_axis_index(const double* k, int n, std::vector<int>& idx, int& nb, double& k0, double& bpu)
{
    nb = 4 * (n - 1);
    const double lo = k[0], hi = k[n - 1];
    const double w = (hi - lo) / nb;
    const double margin = 0.01 * w;
    k0 = lo;
    bpu = 1.0 / w;
    if (!(w > 0.0) || !std::isfinite(bpu) || margin < 1e-12 * std::max(std::fabs(lo), std::fabs(hi)))
        return false;
    for (int b = 0; b < nb; ++b) {
        const int i0 = locate(k, n, lo + b * w - margin);
        const int i1 = locate(k, n, lo + (b + 1) * w + margin);
        if (i1 - i0 > kIndexCompares)
            return false;
        idx.push_back(i0);
    }
    return true;
}

bool aligned(const void* p, uintptr_t bytes)
{
    return (reinterpret_cast<uintptr_t>(p) % bytes) == 0;
}

int grid_for(const pino_ctx* ctx, int64_t n, int block)
{
    const int64_t need = (n + block - 1) / block;
    const int64_t cap = (int64_t)ctx->cu_count * ctx->blocks_per_cu;
    return (int)std::max<int64_t>(1, std::min(need, cap));
}

void free_all(pino_ctx* c)
{
    if (!c)
        return;
    void* ptrs[] = {c->d_growth, c->d_growth32, c->d_gidx, c->d_tknots, c->d_tidx, c->d_tcoef, c->d_tab, c->d_tab32,
                    c->d_tmp, c->d_mlp, c->d_counters, c->d_queue, c->d_kap, c->d_kpoly};
    for (void* p : ptrs)
        if (p)
            (void)hipFree(p);
    c->d_growth = c->d_tknots = c->d_tab = c->d_tmp = nullptr;
    c->d_gidx = nullptr;
    c->d_tidx = nullptr;
    c->d_tcoef = nullptr;
    c->d_tab32 = nullptr;
    c->d_growth32 = nullptr;
    c->d_mlp = nullptr;
    c->d_counters = nullptr;
    c->d_queue = nullptr;
    c->d_kap = nullptr;
    c->d_kpoly = nullptr;
    c->order.destroy();
}

pino_status init_impl(const pino_config* cfg, pino_ctx* c)
{
    PINO_HIP(c, hipSetDevice(cfg->device));
    int cus = 0;
    PINO_HIP(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device));
    c->cu_count = cus > 0 ? cus : 1;
    if (const char* env = std::getenv("PINO_BLOCKS_PER_CU")) {
        const int v = std::atoi(env);
        if (v > 0 && v <= 64)
            c->blocks_per_cu = v;
    }

    // growth tables: [D | a | M] per cosmology, stride 3 * nk_max
    int nk_max = 0;
    for (int k = 0; k < cfg->n_cosmo; ++k)
        nk_max = std::max(nk_max, (int)cfg->growth[k].n);
    c->nk_max = nk_max;
    c->nk.resize(cfg->n_cosmo);
    c->omega.resize(cfg->n_cosmo);
    for (int k = 0; k < cfg->n_cosmo; ++k)
        c->omega[k] = cfg->growth[k].omega_m;
    std::vector<double> host((size_t)cfg->n_cosmo * 3 * nk_max, 0.0);
    for (int k = 0; k < cfg->n_cosmo; ++k) {
        const pino_growth& g = cfg->growth[k];
        c->nk[k] = g.n;
        double* dst = host.data() + (size_t)k * 3 * nk_max;
        std::memcpy(dst, g.D, sizeof(double) * g.n);
        std::memcpy(dst + g.n, g.a, sizeof(double) * g.n);
    }
    PINO_HIP(c, hipMalloc((void**)&c->d_growth, host.size() * sizeof(double)));
    PINO_HIP(c, hipMemcpy(c->d_growth, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));

    // spline scratch: one row per growth table, three per table for the
    // LCDM coefficients
    int64_t tmp_doubles = (int64_t)cfg->n_cosmo * nk_max * (cfg->method == PINO_CLASSIC_LCDM ? 3 : 1);
    if (cfg->method == PINO_TABULATED) {
        const pino_table_knots* t = cfg->table;
        c->nx = t->nx;
        c->ny = t->ny;
        c->nd = t->nd;
        std::vector<double> kn;
        kn.insert(kn.end(), t->x, t->x + t->nx);
        kn.insert(kn.end(), t->y, t->y + t->ny);
        kn.insert(kn.end(), t->delta, t->delta + t->nd);
        PINO_HIP(c, hipMalloc((void**)&c->d_tknots, kn.size() * sizeof(double)));
        PINO_HIP(c, hipMemcpy(c->d_tknots, kn.data(), kn.size() * sizeof(double), hipMemcpyHostToDevice));
        // the interval index, used when all three axes admit it and it fits
        // the LDS budget beside the growth and table knots
        std::vector<int> bins;
        const double* axes[3] = {t->x, t->y, t->delta};
        const int ns[3] = {t->nx, t->ny, t->nd};
        bool ok = true;
        for (int ax = 0; ax < 3 && ok; ++ax)
            ok = table_axis_index(axes[ax], ns[ax], bins, c->tnb[ax], c->tk0[ax], c->tbpu[ax]);
        const size_t lds_need = growth_lds_bytes(nk_max, index_bins(nk_max)) +
                                sizeof(double) * kn.size() + sizeof(int) * bins.size();
        if (ok && lds_need <= kLdsBudget) {
            PINO_HIP(c, hipMalloc((void**)&c->d_tidx, bins.size() * sizeof(int)));
            PINO_HIP(c, hipMemcpy(c->d_tidx, bins.data(), bins.size() * sizeof(int), hipMemcpyHostToDevice));
            c->tindexed = 1;
        }
        // elimination coefficients of the dimensionless delta knots (the row
        // kernels scale them by sigma_R)
        std::vector<double> coef(4 * (size_t)t->nd);
        spline_coef_serial(t->delta, t->nd, coef.data());
        PINO_HIP(c, hipMalloc((void**)&c->d_tcoef, coef.size() * sizeof(double)));
        PINO_HIP(c, hipMemcpy(c->d_tcoef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
        const int64_t cells = (int64_t)t->nx * t->ny * t->nd;
        PINO_HIP(c, hipMalloc((void**)&c->d_tab, 2 * cells * sizeof(double)));
        if (cfg->precision == PINO_MIXED)
            PINO_HIP(c, hipMalloc(&c->d_tab32, (size_t)t->nx * t->ny * (t->nd - 1) * 4 * sizeof(float)));
    }
    PINO_HIP(c, hipMalloc((void**)&c->d_tmp, tmp_doubles * sizeof(double)));

    // natural-spline second derivatives of a(D), built on the device
    for (int k = 0; k < cfg->n_cosmo; ++k) {
        double* g = c->d_growth + (size_t)k * 3 * nk_max;
        const int n = c->nk[k];
        hipLaunchKernelGGL(k_spline_build, dim3(1), dim3(64), 0, 0, g, n, g + n, (int64_t)0, 1, g + 2 * n,
                           (int64_t)0, 1, c->d_tmp + (size_t)k * nk_max, 1);
        PINO_HIP(c, hipGetLastError());
    }

    // LCDM time coefficients at the growth knots and their splines in D
    if (cfg->method == PINO_CLASSIC_LCDM) {
        PINO_HIP(c, hipMalloc((void**)&c->d_kap, (size_t)cfg->n_cosmo * 6 * nk_max * sizeof(double)));
        int* d_nk = nullptr;
        double* d_om = nullptr;
        hipError_t e = hipMalloc((void**)&d_nk, cfg->n_cosmo * sizeof(int));
        if (e == hipSuccess)
            e = hipMalloc((void**)&d_om, cfg->n_cosmo * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpy(d_nk, c->nk.data(), cfg->n_cosmo * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_om, c->omega.data(), cfg->n_cosmo * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_lpt_growth, dim3((cfg->n_cosmo + 63) / 64), dim3(64), 0, 0, c->d_growth, d_nk, d_om,
                               cfg->n_cosmo, nk_max, c->d_kap);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipDeviceSynchronize();
        if (d_nk)
            (void)hipFree(d_nk);
        if (d_om)
            (void)hipFree(d_om);
        PINO_HIP(c, e);
        for (int k = 0; k < cfg->n_cosmo; ++k) {
            double* kp = c->d_kap + (size_t)k * 6 * nk_max;
            const int n = c->nk[k];
            hipLaunchKernelGGL(k_spline_build, dim3(1), dim3(64), 0, 0, c->d_growth + (size_t)k * 3 * nk_max, n, kp,
                               (int64_t)n, 1, kp + 3 * n, (int64_t)n, 1, c->d_tmp + (size_t)k * 3 * nk_max, 3);
            PINO_HIP(c, hipGetLastError());
        }
        // bounds on |d k / d ln D| for the surrogate's certificate: on
        // interval i, |S'| <= |slope_i| + h_i/3 (|M_i| + |M_{i+1}|) and
        // D <= D_{i+1}; outside the knots the ratios are constant
        c->kslope.assign(3 * (size_t)cfg->n_cosmo, 0.0);
        std::vector<double> rows(6 * (size_t)nk_max);
        for (int k = 0; k < cfg->n_cosmo; ++k) {
            const int n = c->nk[k];
            const double* D = cfg->growth[k].D;
            PINO_HIP(c, hipMemcpy(rows.data(), c->d_kap + (size_t)k * 6 * nk_max, 6 * (size_t)n * sizeof(double),
                                  hipMemcpyDeviceToHost));
            for (int j = 0; j < 3; ++j) {
                const double* K = rows.data() + (size_t)j * n;
                const double* M = rows.data() + (size_t)(3 + j) * n;
                double m = 0.0;
                for (int i = 0; i + 1 < n; ++i) {
                    const double h = D[i + 1] - D[i];
                    const double d = std::fabs((K[i + 1] - K[i]) / h) + h / 3.0 * (std::fabs(M[i]) + std::fabs(M[i + 1]));
                    m = std::max(m, D[i + 1] * d);
                }
                c->kslope[3 * (size_t)k + j] = 1.01 * m;
            }
        }
        // the collapse kernels read the power-form coefficients where they
        // fit in LDS (up to about 1200 knots), else the six rows
        const size_t need_poly = lcdm_poly_lds_bytes(nk_max, index_bins(nk_max));
        c->lcdm_poly = need_poly <= kLdsMax;
        if (c->lcdm_poly) {
            const size_t stride = kappa_poly_doubles(nk_max);
            PINO_HIP(c, hipMalloc((void**)&c->d_kpoly, (size_t)cfg->n_cosmo * stride * sizeof(double)));
            for (int k = 0; k < cfg->n_cosmo; ++k) {
                const int n = c->nk[k];
                hipLaunchKernelGGL(k_kappa_poly, dim3((n + 256) / 256), dim3(256), 0, 0,
                                   c->d_growth + (size_t)k * 3 * nk_max, c->d_kap + (size_t)k * 6 * nk_max, n,
                                   c->d_kpoly + (size_t)k * stride);
                PINO_HIP(c, hipGetLastError());
            }
        }
        const size_t need = c->lcdm_poly ? need_poly : lcdm_lds_bytes(nk_max, index_bins(nk_max));
        const void* paired = c->lcdm_poly ? (const void*)k_classic_lcdm<true> : (const void*)k_classic_lcdm<false>;
        const void* single = c->lcdm_poly ? (const void*)k_classic_lcdm_1<true> : (const void*)k_classic_lcdm_1<false>;
        if (need > kLdsBudget) {
            PINO_HIP(c, hipFuncSetAttribute(paired, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
            PINO_HIP(c, hipFuncSetAttribute(single, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need));
        }
        if (const char* env = std::getenv("PINO_LCDM_BLOCK")) {
            const int v = std::atoi(env);
            if (v == 256 || v == 512)
                c->lcdm_block = v;
        }
        int resident = 0;
        PINO_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, paired, c->lcdm_block, need));
        c->lcdm_resident = std::max(1, resident);
    }

    // FP32 copy of the growth knots for the mixed-precision path
    if (cfg->precision == PINO_MIXED) {
        const int64_t count = (int64_t)cfg->n_cosmo * 3 * nk_max;
        PINO_HIP(c, hipMalloc((void**)&c->d_growth32, count * sizeof(float)));
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, 0, c->d_growth,
                           c->d_growth32, count);
        PINO_HIP(c, hipGetLastError());
    }

    // interval index of each growth table (bins uniform in log2 D, up to 4 per
    // knot, kept within the LDS budget of the kernels)
    c->nb_max = index_bins(nk_max);
    c->nb.resize(cfg->n_cosmo);
    c->gL0.resize(cfg->n_cosmo);
    c->gS.resize(cfg->n_cosmo);
    c->gok.resize(cfg->n_cosmo);
    PINO_HIP(c, hipMalloc((void**)&c->d_gidx, (size_t)cfg->n_cosmo * 2 * c->nb_max * sizeof(int)));
    for (int k = 0; k < cfg->n_cosmo; ++k) {
        const pino_growth& g = cfg->growth[k];
        const int nb = index_bins(g.n);
        const float L0 = (float)std::log2(g.D[0]);
        const float S = (float)(nb / (std::log2(g.D[g.n - 1]) - (double)L0));
        c->nb[k] = nb;
        c->gL0[k] = L0;
        c->gS[k] = S;
        int* idx = c->d_gidx + (size_t)k * 2 * c->nb_max;
        hipLaunchKernelGGL(k_growth_index, dim3((nb + 255) / 256), dim3(256), 0, 0, c->d_growth + (size_t)k * 3 * nk_max,
                           g.n, nb, (double)L0, (double)S, idx, idx + c->nb_max);
        PINO_HIP(c, hipGetLastError());
    }
    PINO_HIP(c, hipDeviceSynchronize());
    {
        std::vector<int> need(c->nb_max);
        for (int k = 0; k < cfg->n_cosmo; ++k) {
            PINO_HIP(c, hipMemcpy(need.data(), c->d_gidx + (size_t)k * 2 * c->nb_max + c->nb_max,
                                  c->nb[k] * sizeof(int), hipMemcpyDeviceToHost));
            int worst = 0;
            for (int b = 0; b < c->nb[k]; ++b)
                worst = std::max(worst, need[b]);
            c->gok[k] = worst <= 2 ? 1 : 0;
        }
    }

    if (cfg->precision == PINO_SURROGATE) {
        c->certify_rtol = cfg->certify_rtol > 0.0 ? cfg->certify_rtol : 5e-7;
        pino_status st = mlp_upload(c, cfg->mlp, cfg->mlp_bytes);
        if (st == PINO_OK)
            st = surrogate_lds_limit(c, surrogate_lds_bytes(nk_max, c->nb_max, cfg->method == PINO_CLASSIC_LCDM));
        if (st != PINO_OK)
            return st;
    }
    // evals of a context with per-context scratch are ordered across streams
    if (cfg->method == PINO_TABULATED || cfg->precision == PINO_SURROGATE)
        PINO_HIP(c, c->order.create());
    PINO_HIP(c, hipDeviceSynchronize());
    return PINO_OK;
}

pino_status launch_item(pino_ctx* c, const pino_item& it, uint32_t flags, hipStream_t st)
{
    if (it.n == 0)
        return PINO_OK;
    ItemArgs a;
    for (int k = 0; k < 6; ++k)
        a.h[k] = static_cast<const double*>(it.h[k]);
    a.n = it.n;
    a.nk = c->nk[it.cosmo];
    a.growth = c->d_growth + (size_t)it.cosmo * 3 * c->nk_max;
    a.gi.idx = c->d_gidx + (size_t)it.cosmo * 2 * c->nb_max;
    a.gi.nb = c->nb[it.cosmo];
    a.gi.L0 = c->gL0[it.cosmo];
    a.gi.S = c->gS[it.cosmo];
    a.gi.ok = c->gok[it.cosmo];
    a.radius = it.radius_index;
    a.reset = (flags & PINO_EVAL_RESET) ? 1u : 0u;
    a.finalize = (flags & PINO_EVAL_FINALIZE) ? 1u : 0u;
    a.Fmax = it.Fmax;
    a.Rmax = it.Rmax;
    a.acoll = it.a_coll;
    const int block = 256;
    const size_t lds = growth_lds_bytes(a.nk, a.gi.nb);

    if (c->method == PINO_TABULATED) {
        // per-radius table: F into the interleaved table and the delta
        // splines over the sigma-scaled knots, rebuilt on the device
        const int rows = c->nx * c->ny;
        f4v* pairs = c->precision == PINO_MIXED ? static_cast<f4v*>(c->d_tab32) : nullptr;
        const bool paired_done = launch_table_splines(c->d_tcoef, it.sigma_R, c->nd, it.table_F, c->d_tab, rows, st,
                                                      pairs);
        PINO_HIP(c, hipGetLastError());
        if (pairs && !paired_done) {
            const int64_t count = (int64_t)rows * (c->nd - 1);
            hipLaunchKernelGGL(k_table_pairs_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, c->d_tab,
                               pairs, rows, c->nd);
            PINO_HIP(c, hipGetLastError());
        }
    }

    // the Tabulated kernels' view of the table of this radius
    TabArgs t{};
    if (c->method == PINO_TABULATED) {
        t.xk = c->d_tknots;
        t.yk = c->d_tknots + c->nx;
        t.dk = c->d_tknots + c->nx + c->ny;
        t.nx = c->nx;
        t.ny = c->ny;
        t.nd = c->nd;
        t.scale = it.sigma_R;
        t.inv_scale = 1.0 / it.sigma_R;
        t.tab = c->d_tab;
        t.bidx = c->d_tidx;
        t.indexed = c->tindexed;
        for (int ax = 0; ax < 3; ++ax) {
            t.nb[ax] = c->tnb[ax];
            t.k0[ax] = c->tk0[ax];
            t.bpu[ax] = c->tbpu[ax];
        }
    }

    // the kernels index with 32-bit byte offsets: chunks of at most kChunk
    const size_t esize = c->precision == PINO_MIXED ? sizeof(float) : sizeof(double);
    const ItemArgs a0 = a;
    for (int64_t start = 0; start < a0.n; start += kChunk) {
        a.n = std::min<int64_t>(kChunk, a0.n - start);
        for (int k = 0; k < 6; ++k)
            a.h[k] = reinterpret_cast<const double*>(reinterpret_cast<const char*>(a0.h[k]) + start * esize);
        a.Fmax = a0.Fmax + start;
        a.Rmax = a0.Rmax + start;
        a.acoll = a0.acoll ? a0.acoll + start : nullptr;
        const int g = grid_for(c, a.n, block);
        pino_status ps = PINO_OK;
        if (c->precision == PINO_FP64) {
            // pairs of particles per lane need 16-byte aligned arrays
            bool al = aligned(a.Fmax, 16) && aligned(a.Rmax, 8) && (!a.acoll || aligned(a.acoll, 16));
            for (int k = 0; k < 6; ++k)
                al = al && aligned(a.h[k], 16);
            const int gp = grid_for(c, (a.n + 1) / 2, block);
            if (c->method == PINO_CLASSIC_LCDM) {
                const int lb = c->lcdm_block;
                const int64_t lanes = al ? (a.n + 1) / 2 : a.n;
                const int lg = (int)std::max<int64_t>(
                    1, std::min<int64_t>((lanes + lb - 1) / lb, (int64_t)c->cu_count * c->lcdm_resident));
                if (c->lcdm_poly) {
                    const double* kp = c->d_kpoly + (size_t)it.cosmo * kappa_poly_doubles(c->nk_max);
                    const size_t llds = lcdm_poly_lds_bytes(a.nk, a.gi.nb);
                    if (al)
                        hipLaunchKernelGGL(k_classic_lcdm<true>, dim3(lg), dim3(lb), llds, st, a, kp);
                    else
                        hipLaunchKernelGGL(k_classic_lcdm_1<true>, dim3(lg), dim3(lb), llds, st, a, kp);
                } else {
                    const double* kap = c->d_kap + (size_t)it.cosmo * 6 * c->nk_max;
                    const size_t llds = lcdm_lds_bytes(a.nk, a.gi.nb);
                    if (al)
                        hipLaunchKernelGGL(k_classic_lcdm<false>, dim3(lg), dim3(lb), llds, st, a, kap);
                    else
                        hipLaunchKernelGGL(k_classic_lcdm_1<false>, dim3(lg), dim3(lb), llds, st, a, kap);
                }
            } else if (c->method == PINO_CLASSIC) {
                if (al) {
                    hipLaunchKernelGGL(k_classic_f64, dim3(gp), dim3(block), lds, st, a);
                } else {
                    hipLaunchKernelGGL(k_classic_f64_1, dim3(g), dim3(block), lds, st, a);
                }
            } else {
                const size_t lds_t = lds + table_lds_bytes(t);
                if (al)
                    hipLaunchKernelGGL(k_tabulated_f64, dim3(gp), dim3(block), lds_t, st, a, t);
                else
                    hipLaunchKernelGGL(k_tabulated_f64_1, dim3(g), dim3(block), lds_t, st, a, t);
            }
            PINO_HIP(c, hipGetLastError());
        } else if (c->precision == PINO_MIXED) {
            ps = launch_mixed(c, it, a, c->method == PINO_TABULATED ? &t : nullptr, st, g, block);
        } else {
            ps = launch_surrogate(c, it, a, flags, st, g, block);
        }
        if (ps != PINO_OK)
            return ps;
    }
    return PINO_OK;
}

}  // namespace

extern "C" {

pino_status pino_collapse_init(const pino_config* cfg, pino_ctx** out)
{
    if (!out) {
        g_init_error = "out is NULL";
        return PINO_ERR_ARG;
    }
    *out = nullptr;
    std::string why;
    if (!validate_config(cfg, why)) {
        g_init_error = why;
        return PINO_ERR_ARG;
    }
    if (!lds_fits(cfg, why)) {
        g_init_error = why;
        return PINO_ERR_UNSUPPORTED;
    }
    if (cfg->method == PINO_CLASSIC_LCDM && cfg->precision == PINO_MIXED) {
        g_init_error = "the LCDM method runs in FP64 or with the surrogate, not in mixed precision";
        return PINO_ERR_UNSUPPORTED;
    }
    pino_ctx* c = new (std::nothrow) pino_ctx();
    if (!c) {
        g_init_error = "host allocation failed";
        return PINO_ERR_ALLOC;
    }
    c->device = cfg->device;
    c->method = cfg->method;
    c->precision = cfg->precision;
    c->n_cosmo = cfg->n_cosmo;
    const pino_status st = init_impl(cfg, c);
    if (st != PINO_OK) {
        g_init_error = c->err;
        free_all(c);
        delete c;
        return st;
    }
    *out = c;
    return PINO_OK;
}

pino_status pino_collapse_eval(pino_ctx* ctx, const pino_item* items, int32_t n_items, uint32_t flags,
                               void* hip_stream)
{
    if (!ctx) {
        g_init_error = "ctx is NULL";
        return PINO_ERR_ARG;
    }
    if (ctx->broken) {
        return PINO_ERR_STATE;
    }
    if (flags & ~(PINO_EVAL_RESET | PINO_EVAL_SYNC | PINO_EVAL_FINALIZE)) {
        ctx->err = "unknown flag bits";
        return PINO_ERR_ARG;
    }
    std::string why;
    if (!validate_items(ctx, items, n_items, flags, why)) {
        ctx->err = why;
        return PINO_ERR_ARG;
    }
    PINO_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    PINO_HIP(ctx, ctx->order.enter(st));
    for (int32_t k = 0; k < n_items; ++k) {
        const pino_status s = launch_item(ctx, items[k], flags, st);
        if (s != PINO_OK)
            return s;
    }
    PINO_HIP(ctx, ctx->order.leave(st));
    if (flags & PINO_EVAL_SYNC)
        PINO_HIP(ctx, hipStreamSynchronize(st));
    return PINO_OK;
}

pino_status pino_collapse_free(pino_ctx* ctx)
{
    if (!ctx)
        return PINO_OK;
    pino_status st = PINO_OK;
    if (hipSetDevice(ctx->device) == hipSuccess) {
        if (hipDeviceSynchronize() != hipSuccess)
            st = PINO_ERR_HIP;
    }
    free_all(ctx);
    delete ctx;
    return st;
}

const char* pino_collapse_last_error(const pino_ctx* ctx)
{
    if (!ctx)
        return g_init_error.c_str();
    return ctx->err.c_str();
}

pino_status pino_collapse_ellipsoid_table_mg(pino_ctx* ctx, int32_t cosmo, double sigma_R, double mu0,
                                             double* table_F, void* hip_stream)
{
    if (!ctx) {
        g_init_error = "ctx is NULL";
        return PINO_ERR_ARG;
    }
    if (ctx->broken)
        return PINO_ERR_STATE;
    if (ctx->method != PINO_TABULATED || cosmo < 0 || cosmo >= ctx->n_cosmo || !table_F ||
        !(std::isfinite(sigma_R) && sigma_R > 0.0)) {
        ctx->err = "need a PINO_TABULATED context, a valid cosmology index, a finite sigma_R > 0 and table_F";
        return PINO_ERR_ARG;
    }
    const double om = ctx->omega[cosmo];
    if (!(om > 0.0 && om <= 1.0)) {
        ctx->err = "the ellipsoid table needs 0 < omega_m <= 1 (flat, no radiation)";
        return PINO_ERR_ARG;
    }
    // mu(a) = 1 + mu0 / E^2 stays positive for mu0 > -(1 - omega_m); without
    // a cosmological constant 1/E^2 = a^3 grows without bound, so only 0
    if (!std::isfinite(mu0) || (om < 1.0 ? !(mu0 > -(1.0 - om)) : mu0 != 0.0)) {
        ctx->err = "mu0 must be finite and > -(1 - omega_m) (and 0 when omega_m = 1)";
        return PINO_ERR_ARG;
    }
    PINO_HIP(ctx, hipSetDevice(ctx->device));
    double D1;
    if (mu0 == 0.0) {
        if (ctx->ell_D1.empty())
            ctx->ell_D1.assign(ctx->n_cosmo, 0.0);
        if (!(ctx->ell_D1[cosmo] > 0.0))
            ctx->ell_D1[cosmo] = ell_growth_today(om, 0.0);
        D1 = ctx->ell_D1[cosmo];
    } else {
        D1 = ell_growth_today(om, mu0);  // a few ms on the host
    }
    const int64_t nodes = (int64_t)ctx->nx * ctx->ny * ctx->nd;
    hipLaunchKernelGGL(k_ellipsoid_table, dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), ctx->d_tknots, ctx->nx, ctx->ny, ctx->nd, sigma_R, om,
                       mu0, D1, table_F);
    PINO_HIP(ctx, hipGetLastError());
    return PINO_OK;
}

pino_status pino_collapse_ellipsoid_table(pino_ctx* ctx, int32_t cosmo, double sigma_R, double* table_F,
                                          void* hip_stream)
{
    return pino_collapse_ellipsoid_table_mg(ctx, cosmo, sigma_R, 0.0, table_F, hip_stream);
}

pino_status pino_collapse_lpt_coefficients(pino_ctx* ctx, int32_t cosmo, double* k2, double* k3a, double* k3b)
{
    if (!ctx) {
        g_init_error = "ctx is NULL";
        return PINO_ERR_ARG;
    }
    if (ctx->broken)
        return PINO_ERR_STATE;
    if (ctx->method != PINO_CLASSIC_LCDM || cosmo < 0 || cosmo >= ctx->n_cosmo || !k2 || !k3a || !k3b) {
        ctx->err = "need a PINO_CLASSIC_LCDM context, a valid cosmology index and non-NULL outputs";
        return PINO_ERR_ARG;
    }
    PINO_HIP(ctx, hipSetDevice(ctx->device));
    PINO_HIP(ctx, hipDeviceSynchronize());
    const int n = ctx->nk[cosmo];
    const double* src = ctx->d_kap + (size_t)cosmo * 6 * ctx->nk_max;
    PINO_HIP(ctx, hipMemcpy(k2, src, n * sizeof(double), hipMemcpyDeviceToHost));
    PINO_HIP(ctx, hipMemcpy(k3a, src + n, n * sizeof(double), hipMemcpyDeviceToHost));
    PINO_HIP(ctx, hipMemcpy(k3b, src + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost));
    return PINO_OK;
}

}  // extern "C"

extern "C" {

pino_status pino_collapse_features(pino_ctx* ctx, const pino_item* item, float* x, float* w, void* hip_stream)
{
    if (!ctx || !item || (item->n > 0 && !x)) {
        g_init_error = "ctx, item and x must be non-NULL";
        return PINO_ERR_ARG;
    }
    if (ctx->broken)
        return PINO_ERR_STATE;
    std::string why;
    pino_item it = *item;
    double* dummyF = reinterpret_cast<double*>(x);  // outputs are not written; validation wants them non-NULL
    if (!it.Fmax)
        it.Fmax = dummyF;
    if (!it.Rmax)
        it.Rmax = reinterpret_cast<int32_t*>(x);
    if (!validate_items(ctx, &it, 1, 0, why)) {
        ctx->err = why;
        return PINO_ERR_ARG;
    }
    if (!(std::isfinite(it.sigma_R) && it.sigma_R > 0.0)) {
        ctx->err = "sigma_R must be finite and > 0";
        return PINO_ERR_ARG;
    }
    if (it.n > kChunk) {
        ctx->err = "pino_collapse_features takes at most 2^28 particles per call";
        return PINO_ERR_ARG;
    }
    if (it.n == 0)
        return PINO_OK;
    PINO_HIP(ctx, hipSetDevice(ctx->device));
    ItemArgs a{};
    for (int k = 0; k < 6; ++k)
        a.h[k] = static_cast<const double*>(it.h[k]);
    a.n = it.n;
    // the growth knots and index (global memory) for the LCDM ratio splines
    a.nk = ctx->nk[it.cosmo];
    a.growth = ctx->d_growth + (size_t)it.cosmo * 3 * ctx->nk_max;
    a.gi.idx = ctx->d_gidx + (size_t)it.cosmo * 2 * ctx->nb_max;
    a.gi.nb = ctx->nb[it.cosmo];
    a.gi.L0 = ctx->gL0[it.cosmo];
    a.gi.S = ctx->gS[it.cosmo];
    a.gi.ok = ctx->gok[it.cosmo];
    const double* kap =
        ctx->method == PINO_CLASSIC_LCDM ? ctx->d_kap + (size_t)it.cosmo * 6 * ctx->nk_max : nullptr;
    const bool f32 = ctx->precision == PINO_MIXED;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((it.n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), a, f32, it.sigma_R, ctx->omega[it.cosmo], kap, x, w);
    PINO_HIP(ctx, hipGetLastError());
    return PINO_OK;
}

pino_status pino_collapse_predict(pino_ctx* ctx, const float* x, float* y, int64_t n, void* hip_stream)
{
    if (!ctx || n < 0 || (n > 0 && (!x || !y))) {
        g_init_error = "bad arguments";
        return PINO_ERR_ARG;
    }
    if (ctx->broken)
        return PINO_ERR_STATE;
    if (ctx->precision != PINO_SURROGATE) {
        ctx->err = "pino_collapse_predict needs a PINO_SURROGATE context";
        return PINO_ERR_ARG;
    }
    if (n == 0)
        return PINO_OK;
    PINO_HIP(ctx, hipSetDevice(ctx->device));
    const int grid = grid_for(ctx, n, 256);
    hipLaunchKernelGGL(k_predict, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                       static_cast<const NetFrags*>(ctx->d_mlp), x, y, n);
    PINO_HIP(ctx, hipGetLastError());
    return PINO_OK;
}

pino_status pino_collapse_surrogate_stats(pino_ctx* ctx, int64_t* certified, int64_t* fallback,
                                          int64_t* gated_solved, int64_t* gated_zero, int32_t reset)
{
    if (!ctx) {
        g_init_error = "ctx is NULL";
        return PINO_ERR_ARG;
    }
    if (ctx->broken)
        return PINO_ERR_STATE;
    if (ctx->precision != PINO_SURROGATE || !ctx->d_counters) {
        ctx->err = "surrogate statistics need a PINO_SURROGATE context";
        return PINO_ERR_ARG;
    }
    PINO_HIP(ctx, hipSetDevice(ctx->device));
    PINO_HIP(ctx, hipDeviceSynchronize());
    // four counters per block slot of the surrogate kernel, summed here
    std::vector<int64_t> slots(4 * (size_t)kQueueBlocks);
    PINO_HIP(ctx, hipMemcpy(slots.data(), ctx->d_counters, slots.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    int64_t v[4] = {0, 0, 0, 0};
    for (size_t b = 0; b < slots.size(); b += 4)
        for (int k = 0; k < 4; ++k)
            v[k] += slots[b + k];
    if (certified)
        *certified = v[0];
    if (fallback)
        *fallback = v[1];
    if (gated_solved)
        *gated_solved = v[2];
    if (gated_zero)
        *gated_zero = v[3];
    if (reset)
        PINO_HIP(ctx, hipMemset(ctx->d_counters, 0, slots.size() * sizeof(int64_t)));
    return PINO_OK;
}

}  // extern "C"

#include "batch_api.h"
#include "field_api.h"
#include "interp_api.h"
