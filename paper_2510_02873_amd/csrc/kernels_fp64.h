// FP64 kernels of the collapse-time path: spline construction (Classic growth
// tables and the per-radius delta splines of the Tabulated method) and the
// per-radius collapse + max-update kernels.
#pragma once

#include "device_collapse.h"

namespace pino {

// ---------------------------------------------------------------------------
// Spline construction (Sec. 4.2: the interpolation tables are built on the
// device so the per-radius Tabulated update never goes through the host).
// Natural cubic spline second derivatives for `rows` value rows over shared
// knots x[0..n-1]:
//   h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
//     = 6 [(y_{i+1} - y_i)/h_i - (y_i - y_{i-1})/h_{i-1}],  M_0 = M_{n-1} = 0,
// one Thomas solve per thread.  Row r reads y[r*ldy + k*sy] and writes
// m[r*ldm + k*sm]; `tmp` holds n doubles per row (the eliminated
// super-diagonal).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_spline_build(const double* __restrict__ x, int n, const double* __restrict__ y,
                                                    int64_t ldy, int sy, double* __restrict__ m, int64_t ldm, int sm,
                                                    double* __restrict__ tmp, int rows)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows)
        return;
    const double* yr = y + r * ldy;
    double* mr = m + r * ldm;
    double* cp = tmp + (int64_t)r * n;
    mr[0] = 0.0;
    mr[(int64_t)(n - 1) * sm] = 0.0;
    if (n < 3)
        return;
    // forward sweep over unknowns i = 1..n-2 (d' kept in m, c' in tmp)
    double cprev = 0.0, dprev = 0.0;
    double hl = x[1] - x[0];
    double yl = yr[0], yc = yr[sy];
    for (int i = 1; i <= n - 2; ++i) {
        const double hr = x[i + 1] - x[i];
        const double yn = yr[(int64_t)(i + 1) * sy];
        const double rhs = 6.0 * ((yn - yc) / hr - (yc - yl) / hl);
        const double den = 2.0 * (hl + hr) - hl * cprev;
        const double c = hr / den;
        const double d = (rhs - hl * dprev) / den;
        cp[i] = c;
        mr[(int64_t)i * sm] = d;
        cprev = c;
        dprev = d;
        hl = hr;
        yl = yc;
        yc = yn;
    }
    // back substitution
    double mnext = 0.0;
    for (int i = n - 2; i >= 1; --i) {
        const double v = mr[(int64_t)i * sm] - cp[i] * mnext;
        mr[(int64_t)i * sm] = v;
        mnext = v;
    }
}

// ---------------------------------------------------------------------------
// Table splines (the per-radius rebuild of the Tabulated method): every
// delta row of the table shares the knots, so the elimination coefficients
// of the system above are computed once and each row then needs only
// multiplies and adds.  For unknown i (1 <= i <= n-2), with
// h_i = x_{i+1} - x_i:
//   den_i = 2 (h_{i-1} + h_i) - h_{i-1} c_{i-1},  c_i = h_i / den_i (c_0 = 0),
//   coef[4i .. 4i+3] = {1/h_i, h_{i-1}, 1/den_i, c_i};  coef[0] = 1/h_0.
// Under x -> s x, 1/h and 1/den scale by 1/s, h by s, and c is unchanged, so
// a context keeps the coefficients of its dimensionless knots and the row
// kernels apply sigma_R.
// ---------------------------------------------------------------------------
__host__ __device__ inline void spline_coef_serial(const double* x, int n, double* coef)
{
    double xc = x[1];
    double hl = xc - x[0];
    coef[0] = 1.0 / hl;
    coef[1] = coef[2] = coef[3] = 0.0;
    double cprev = 0.0;
    for (int i = 1; i <= n - 2; ++i) {
        const double xn = x[i + 1];
        const double hr = xn - xc;
        const double iden = 1.0 / (2.0 * (hl + hr) - hl * cprev);
        const double c = hr * iden;
        coef[4 * i + 0] = 1.0 / hr;
        coef[4 * i + 1] = hl;
        coef[4 * i + 2] = iden;
        coef[4 * i + 3] = c;
        cprev = c;
        hl = hr;
        xc = xn;
    }
}

// The coefficients of the knots xk[k] * scale on the device (one wave: the
// knots are staged in LDS, at most kCoefKnots; lane 0 runs the recurrence).
constexpr int kCoefKnots = 4096;

__global__ void __launch_bounds__(64) k_spline_coef(const double* __restrict__ xk, int n, double scale,
                                                   double* __restrict__ coef)
{
    __shared__ double xs[kCoefKnots];
    if (blockIdx.x != 0)
        return;
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        xs[k] = xk[k] * scale;
    __syncthreads();
    if (threadIdx.x == 0)
        spline_coef_serial(xs, n, coef);
}

// Row r of F ([rows][n]) into the interleaved table: tab[2 (r n + k)] = F,
// tab[2 (r n + k) + 1] = M_k, knots scaled by s (inv_s = 1/s) from the
// coefficients above.  One row per lane: forward elimination
//   d_i = (6 [(y_{i+1} - y_i)/h_i - (y_i - y_{i-1})/h_{i-1}] - h_{i-1} d_{i-1}) / den_i
// (d_i stored in the M slot), then back substitution M_i = d_i - c_i M_{i+1}.
// The row's values are read kSplineBatch at a time so their loads overlap;
// the coefficients are wave-uniform loads.  Used for rows longer than
// k_table_splines_scan takes.
constexpr int kSplineBatch = 32;

__global__ void __launch_bounds__(64) k_table_splines(const double* __restrict__ coef, double s, double inv_s,
                                                     int n, const double* __restrict__ F, double* __restrict__ tab,
                                                     int rows)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows)
        return;
    const double* y = F + (int64_t)r * n;
    double* t = tab + (int64_t)r * n * 2;
    const double y0 = y[0];
    double yc = y[1];
    t[0] = y0;
    t[1] = 0.0;
    double sl = (yc - y0) * (coef[0] * inv_s);  // slope of the interval left of unknown i
    double dprev = 0.0;
    for (int i0 = 1; i0 <= n - 2; i0 += kSplineBatch) {
        double yn[kSplineBatch];
#pragma unroll
        for (int k = 0; k < kSplineBatch; ++k)
            yn[k] = i0 + k + 1 < n ? y[i0 + k + 1] : 0.0;
#pragma unroll
        for (int k = 0; k < kSplineBatch; ++k) {
            const int i = i0 + k;
            if (i <= n - 2) {
                const double* cf = coef + 4 * i;
                const double sr = (yn[k] - yc) * (cf[0] * inv_s);
                const double d = (6.0 * (sr - sl) - (cf[1] * s) * dprev) * (cf[2] * inv_s);
                t[2 * i] = yc;
                t[2 * i + 1] = d;
                dprev = d;
                sl = sr;
                yc = yn[k];
            }
        }
    }
    t[2 * (n - 1)] = yc;
    t[2 * (n - 1) + 1] = 0.0;
    double mnext = 0.0;
    for (int i0 = n - 2; i0 >= 1; i0 -= kSplineBatch) {
        double dv[kSplineBatch];
#pragma unroll
        for (int k = 0; k < kSplineBatch; ++k)
            dv[k] = i0 - k >= 1 ? t[2 * (i0 - k) + 1] : 0.0;
#pragma unroll
        for (int k = 0; k < kSplineBatch; ++k) {
            const int i = i0 - k;
            if (i >= 1) {
                const double v = dv[k] - coef[4 * i + 3] * mnext;
                t[2 * i + 1] = v;
                mnext = v;
            }
        }
    }
}

// The same system with one wave per row (n <= 64 kScanPer): lane L holds the
// m = ceil(n / 64) consecutive knots i = L m .. L m + m - 1.  Both
// recurrences are affine, d_i = A_i d_{i-1} + B_i with A_i = -h_{i-1}/den_i,
// B_i = 6 (slope_i - slope_{i-1})/den_i, and M_i = -c_i M_{i+1} + d_i, so
// each lane composes its own maps, a wave scan (6 shuffle steps) composes
// the lanes' maps, and each lane then applies its maps from the value the
// scan hands it.  |A_i| and |c_i| are below 1 (diagonal dominance), so the
// composed maps stay bounded; the result differs from the sequential
// elimination by rounding only.
constexpr int kScanPer = 8;

typedef float f4v __attribute__((ext_vector_type(4)));

// inclusive scan of x -> A x + B over lanes 0..L (up) or L..63 (down);
// the map of the nearer lanes is applied last
__device__ __forceinline__ void affine_scan(double& A, double& B, int lane, bool up)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double Ao = up ? __shfl_up(A, off, 64) : __shfl_down(A, off, 64);
        const double Bo = up ? __shfl_up(B, off, 64) : __shfl_down(B, off, 64);
        if (up ? lane >= off : lane + off < 64) {
            B = fma(A, Bo, B);
            A = A * Ao;
        }
    }
}

// pairs (may be NULL): also write the FP32 knot-pair copy of the row,
// pairs[r (n - 1) + i] = (F_i, M_i, F_{i+1}, M_{i+1}), i < n - 1, the values
// rounded from the FP64 ones written to tab.
__global__ void __launch_bounds__(256) k_table_splines_scan(const double* __restrict__ coef, double s, double inv_s,
                                                           int n, const double* __restrict__ F,
                                                           double* __restrict__ tab, int rows,
                                                           f4v* __restrict__ pairs)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= rows)
        return;  // the whole wave
    const int m = (n + 63) >> 6;
    const int i0 = lane * m;
    const double* y = F + (int64_t)r * n;
    double* t = tab + (int64_t)r * n * 2;
    double yv[kScanPer], A[kScanPer], B[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        yv[k] = (k < m && i0 + k < n) ? y[i0 + k] : 0.0;
    // slopes of intervals i0 + k, and the slope left of i0 from lane - 1
    const double ynl = __shfl_down(yv[0], 1, 64);  // first knot of the next lane
    double sv[kScanPer];
    double slast = 0.0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = i0 + k;
        double yn = ynl;
#pragma unroll
        for (int q = k + 1; q < kScanPer; ++q)
            yn = q == k + 1 && q < m ? yv[q] : yn;
        sv[k] = (k < m && i <= n - 2) ? (yn - yv[k]) * (coef[4 * i] * inv_s) : 0.0;
        slast = k < m ? sv[k] : slast;
    }
    const double sprev_lane = __shfl_up(slast, 1, 64);
    // forward maps, composed over the lane's knots
    double Al = 1.0, Bl = 0.0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = i0 + k;
        double a = 1.0, b = 0.0;
        if (k < m && i == 0) {
            a = 0.0;
        } else if (k < m && i <= n - 2) {
            const double iden = coef[4 * i + 2] * inv_s;
            const double sl = k == 0 ? sprev_lane : sv[k > 0 ? k - 1 : 0];
            a = -(coef[4 * i + 1] * s) * iden;
            b = 6.0 * (sv[k] - sl) * iden;
        }
        A[k] = a;
        B[k] = b;
        Bl = fma(a, Bl, b);
        Al = a * Al;
    }
    affine_scan(Al, Bl, lane, true);
    double d = __shfl_up(Bl, 1, 64);  // d just before the lane's first knot
    if (lane == 0)
        d = 0.0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        d = fma(A[k], d, B[k]);
        B[k] = d;  // d_i
    }
    // backward maps M_i = -c_i M_{i+1} + d_i (0 at i = 0 and i >= n - 1)
    Al = 1.0;
    Bl = 0.0;
#pragma unroll
    for (int k = kScanPer - 1; k >= 0; --k) {
        const int i = i0 + k;
        double a = 1.0, b = 0.0;
        if (k < m) {
            if (i >= 1 && i <= n - 2) {
                a = -coef[4 * i + 3];
                b = B[k];
            } else {
                a = 0.0;
            }
        }
        A[k] = a;
        B[k] = b;
        Bl = fma(a, Bl, b);
        Al = a * Al;
    }
    affine_scan(Al, Bl, lane, false);
    double M = __shfl_down(Bl, 1, 64);  // M just after the lane's last knot
    if (lane == 63)
        M = 0.0;
    f4v* pr = pairs ? pairs + (int64_t)r * (n - 1) : nullptr;
#pragma unroll
    for (int k = kScanPer - 1; k >= 0; --k) {
        const double Mn = M;  // M of the next knot (steps k >= m are identities)
        M = fma(A[k], M, B[k]);
        const int i = i0 + k;
        if (k < m && i < n) {
            t[2 * i] = yv[k];
            t[2 * i + 1] = M;
            if (pr && i <= n - 2) {
                double yn = ynl;
#pragma unroll
                for (int q = k + 1; q < kScanPer; ++q)
                    yn = q == k + 1 && q < m ? yv[q] : yn;
                pr[i] = f4v{(float)yv[k], (float)M, (float)yn, (float)Mn};
            }
        }
    }
}

// The table splines of `rows` rows of n knots scaled by s (coef as above):
// one wave per row when the row fits the scan kernel, else one row per lane.
// Returns whether the FP32 knot-pair copy (pairs, may be NULL) was written
// too (the scan kernel writes it in the same pass).
inline bool launch_table_splines(const double* coef, double s, int n, const double* F, double* tab, int rows,
                                 hipStream_t st, f4v* pairs = nullptr)
{
    if (n <= 64 * kScanPer) {
        hipLaunchKernelGGL(k_table_splines_scan, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, coef, s,
                           1.0 / s, n, F, tab, rows, pairs);
        return pairs != nullptr;
    }
    hipLaunchKernelGGL(k_table_splines, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0, st, coef, s, 1.0 / s, n,
                       F, tab, rows);
    return false;
}

// ---------------------------------------------------------------------------
// Per-radius Classic FP64 kernel.  One particle per lane per step of a
// grid-stride loop; the growth knots [D | a | M] of the item's cosmology are
// staged once per workgroup in LDS.  Hessian loads are coalesced SoA reads
// that bypass the caches' retention (each value is read once).
// ---------------------------------------------------------------------------
// Items reach the per-radius kernels in chunks of at most kChunk particles,
// so that an element's byte offset i * sizeof(T) fits in 32 bits: loads and
// stores then take the scalar-base + 32-bit vector-offset form, one offset
// shared by every array with the same element size.
constexpr int64_t kChunk = int64_t(1) << 28;

struct ItemArgs {
    const double* h[6];
    int64_t n;                // <= kChunk in the per-radius kernels
    const double* growth;  // [D | a | M], nk each
    int nk;
    GrowthIndex gi;        // idx points to global memory; kernels stage it
    int32_t radius;
    uint32_t reset;
    uint32_t finalize;
    double* Fmax;
    int32_t* Rmax;
    double* acoll;
};

template <typename T>
__device__ __forceinline__ const T* elem(const T* base, uint32_t i)
{
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ T* elem(T* base, uint32_t i)
{
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T));
}

__device__ __forceinline__ void stage(double* dst, const double* __restrict__ src, int count)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x)
        dst[k] = src[k];
}

// growth knots and their interval index into LDS; returns the LDS index view
__device__ __forceinline__ GrowthIndex stage_growth(double* lds, const ItemArgs& a)
{
    stage(lds, a.growth, 3 * a.nk);
    int* idx = reinterpret_cast<int*>(lds + 3 * a.nk);
    for (int k = threadIdx.x; k < a.gi.nb; k += blockDim.x)
        idx[k] = a.gi.idx[k];
    GrowthIndex gi = a.gi;
    gi.idx = idx;
    return gi;
}

// LDS bytes of stage_growth
__host__ __device__ inline size_t growth_lds_bytes(int nk, int nb)
{
    return 3 * (size_t)nk * sizeof(double) + (((size_t)nb * sizeof(int) + 7) / 8) * 8;
}

__device__ __forceinline__ Hess64 load_h64(const ItemArgs& a, uint32_t i)
{
    Hess64 h;
    h.xx = __builtin_nontemporal_load(elem(a.h[0], i));
    h.yy = __builtin_nontemporal_load(elem(a.h[1], i));
    h.zz = __builtin_nontemporal_load(elem(a.h[2], i));
    h.xy = __builtin_nontemporal_load(elem(a.h[3], i));
    h.xz = __builtin_nontemporal_load(elem(a.h[4], i));
    h.yz = __builtin_nontemporal_load(elem(a.h[5], i));
    return h;
}

// Max update with the strict '>' rule.  Every element is written, whether
// or not its maximum changes: a wave then stores whole cache lines, which HBM
// takes far faster than the partial lines of masked stores (the old Rmax and
// a_coll are read to be written back).  a(D_c), D_c = 1/F, is evaluated only
// where needed: on update, or for every element from the running maximum
// when finalizing.
__device__ __forceinline__ void update_max(const ItemArgs& a, const double* g, const GrowthIndex& gi, uint32_t i,
                                           double F, double fm)
{
    const bool upd = F > fm;
    const double fnew = upd ? F : fm;
    const int32_t rm = a.reset ? -1 : *elem(a.Rmax, i);
    *elem(a.Fmax, i) = fnew;
    *elem(a.Rmax, i) = upd ? a.radius : rm;
    if (a.acoll) {
        double* ac = elem(a.acoll, i);
        if (a.finalize) {
            *ac = fnew > 0.0 ? growth_invert(g, a.nk, rcp2(fnew), gi) : kInf;
        } else {
            const double am = a.reset ? kInf : *ac;
            *ac = upd ? growth_invert(g, a.nk, rcp2(F), gi) : am;
        }
    }
}

#ifndef PINO_WAVES_PER_EU
#define PINO_WAVES_PER_EU 4
#endif

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PINO_WAVES_PER_EU)))
k_classic_f64_1(ItemArgs a)
{
    extern __shared__ double lds[];
    const GrowthIndex gi = stage_growth(lds, a);
    __syncthreads();
    // One particle per lane (arrays not 16-byte aligned).  Software pipeline:
    // the loads of the next grid-stride element are issued before the
    // eigen/root arithmetic of the current one, so their latency hides
    // behind it.
    const uint32_t n = (uint32_t)a.n;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    Hess64 hn{};
    double fn = 0.0;
    if (i < n) {
        hn = load_h64(a, i);
        fn = a.reset ? 0.0 : *elem(a.Fmax, i);
    }
    for (; i < n; i += stride) {
        const Hess64 h = hn;
        const double fm = fn;
        const uint32_t next = i + stride;
        if (next < n) {
            hn = load_h64(a, next);
            fn = a.reset ? 0.0 : *elem(a.Fmax, next);
        }
        double l1, s, pp;
        eig_top(h, l1, s, pp);
        const double F = classic_F(l1, s, pp);
        update_max(a, lds, gi, i, F, fm);
    }
}

typedef double d2v __attribute__((ext_vector_type(2)));

// Two adjacent particles per lane: one 16-byte load per Hessian component
// (and per output array) instead of two 8-byte ones.
struct Hess2 {
    d2v xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ Hess2 load_h2(const ItemArgs& a, uint32_t p)
{
    Hess2 h;
    h.xx = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(elem(a.h[0], 2 * p)));
    h.yy = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(elem(a.h[1], 2 * p)));
    h.zz = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(elem(a.h[2], 2 * p)));
    h.xy = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(elem(a.h[3], 2 * p)));
    h.xz = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(elem(a.h[4], 2 * p)));
    h.yz = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(elem(a.h[5], 2 * p)));
    return h;
}

// update_max for the pair (2p, 2p + 1), element for element, with paired
// (whole-line) loads and stores
__device__ __forceinline__ void update_pair(const ItemArgs& a, const double* g, const GrowthIndex& gi, uint32_t p,
                                            double F0, double F1, d2v fm)
{
    const bool u0 = F0 > fm.x, u1 = F1 > fm.y;
    const d2v fnew{u0 ? F0 : fm.x, u1 ? F1 : fm.y};
    int2 rm{-1, -1};
    if (!a.reset)
        rm = *reinterpret_cast<const int2*>(elem(a.Rmax, 2 * p));
    *reinterpret_cast<d2v*>(elem(a.Fmax, 2 * p)) = fnew;
    *reinterpret_cast<int2*>(elem(a.Rmax, 2 * p)) = int2{u0 ? a.radius : rm.x, u1 ? a.radius : rm.y};
    if (a.acoll) {
        d2v* ac = reinterpret_cast<d2v*>(elem(a.acoll, 2 * p));
        d2v v;
        if (a.finalize) {
            v.x = fnew.x > 0.0 ? growth_invert(g, a.nk, rcp2(fnew.x), gi) : kInf;
            v.y = fnew.y > 0.0 ? growth_invert(g, a.nk, rcp2(fnew.y), gi) : kInf;
        } else {
            const d2v am = a.reset ? d2v{kInf, kInf} : *ac;
            v.x = u0 ? growth_invert(g, a.nk, rcp2(F0), gi) : am.x;
            v.y = u1 ? growth_invert(g, a.nk, rcp2(F1), gi) : am.y;
        }
        *ac = v;
    }
}

__device__ __forceinline__ double classic_of(const Hess64& h)
{
    double l1, s, pp;
    eig_top(h, l1, s, pp);
    return classic_F(l1, s, pp);
}

// The headline kernel: pairs (2p, 2p + 1) over a grid-stride loop, the next
// pair's loads issued before the current pair's arithmetic; the update is
// update_max's, element for element, with whole-line paired stores.  Needs
// 16-byte aligned Hessian, Fmax and a_coll arrays and an 8-byte aligned Rmax
// (checked by the host); an odd last element is done by one lane at the end.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PINO_WAVES_PER_EU)))
k_classic_f64(ItemArgs a)
{
    extern __shared__ double lds[];
    const GrowthIndex gi = stage_growth(lds, a);
    __syncthreads();
    const uint32_t n = (uint32_t)a.n;
    const uint32_t np = n / 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    Hess2 hn{};
    d2v fn{0.0, 0.0};
    if (p < np) {
        hn = load_h2(a, p);
        if (!a.reset)
            fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * p));
    }
    for (; p < np; p += stride) {
        const Hess2 h = hn;
        const d2v fm = fn;
        const uint32_t next = p + stride;
        if (next < np) {
            hn = load_h2(a, next);
            if (!a.reset)
                fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * next));
        }
        const double F0 = classic_of(Hess64{h.xx.x, h.yy.x, h.zz.x, h.xy.x, h.xz.x, h.yz.x});
        const double F1 = classic_of(Hess64{h.xx.y, h.yy.y, h.zz.y, h.xy.y, h.xz.y, h.yz.y});
        update_pair(a, lds, gi, p, F0, F1, fm);
    }
    if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t i = n - 1;
        const double fm = a.reset ? 0.0 : *elem(a.Fmax, i);
        update_max(a, lds, gi, i, classic_of(load_h64(a, i)), fm);
    }
}

// ---------------------------------------------------------------------------
// Tabulated FP64.  The library keeps, per radius, an interleaved copy of the
// table, tab[((ix*ny + iy)*nd + id)*2 + {0,1}] = (F, M), so the two knots of a
// corner spline are 32 contiguous bytes.  Knots (scaled by sigma_R) live in
// LDS after the growth knots, followed by the per-axis interval index.
//
// Interval index (per axis, optional): nb uniform bins over the dimensionless
// knot range; bin b holds the interval `locate` returns at the bin's low end
// less a margin of 1 % of a bin, and the host has verified that at most
// kIndexCompares more knots lie below the bin's high end plus the margin, so
// that many compares (whose knot reads are independent) finish the search.  The margin is far
// above the rounding of the bin arithmetic, and the interval found is the one
// `locate` finds.  Without the index (indexed = 0) the binary search is used.
// ---------------------------------------------------------------------------
struct TabArgs {
    const double* xk;  // dimensionless knots, nx, ny, nd
    const double* yk;
    const double* dk;
    int nx, ny, nd;
    double scale;      // sigma_R
    double inv_scale;  // 1 / sigma_R
    const double* tab; // interleaved (F, M)
    const int* bidx;   // interval index bins, x | y | delta (nb[0] + nb[1] + nb[2])
    int nb[3];
    double k0[3];      // first dimensionless knot per axis
    double bpu[3];     // bins per dimensionless unit
    int indexed;
};

// Interval of the scaled knots xs (n) containing q: `locate`, through the
// axis index when there is one.
// Finish an interval search from interval i: up to K more knots, read
// independently of each other.  The Tabulated kernels' table index allows
// kIndexCompares (smooth knots, checked by the host); the stand-alone
// spline's per-block index allows one more (random knots cluster).
constexpr int kIndexCompares = 2;

template <int K = kIndexCompares>
__host__ __device__ __forceinline__ int locate_after(const double* xs, int n, double q, int i)
{
    double xv[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        xv[k] = xs[min(i + 1 + k, n - 1)];
    int r = i, c = 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        c = c & ((i + 1 + k <= n - 2 && xv[k] <= q) ? 1 : 0);
        r += c;
    }
    return r;
}

__host__ __device__ __forceinline__ int table_locate(const TabArgs& t, int axis, const int* idx, const double* xs, int n,
                                            double q)
{
    if (!t.indexed)
        return locate(xs, n, q);
    double fb = (q * t.inv_scale - t.k0[axis]) * t.bpu[axis];
    fb = fmin(fmax(fb, 0.0), (double)(t.nb[axis] - 1));
    return locate_after(xs, n, q, idx[(int)fb]);
}

// The interval index of knots xs[0..n-1] (LDS), built by the whole block:
// nb uniform bins over [xs[0], xs[n-1]], bin b holding the interval at its
// low end less a margin of 1 % of a bin.  Returns, the same on every thread,
// whether at most K more knots follow inside any bin (margins included) and
// the margin is far above the rounding of the bin arithmetic; bpu receives
// the bins per unit.  All threads of the block must call it.
template <int K>
__device__ __forceinline__ bool build_axis_index(const double* xs, int n, int nb, int* idx, double& bpu)
{
    const double lo = xs[0], hi = xs[n - 1];
    const double w = (hi - lo) / nb;
    bpu = 1.0 / w;
    bool ok = w > 0.0 && isfinite(bpu) && 0.01 * w >= 1e-12 * fmax(fabs(lo), fabs(hi));
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const int i0 = locate(xs, n, lo + (b - 0.01) * w);
        const int i1 = locate(xs, n, lo + (b + 1.01) * w);
        idx[b] = i0;
        ok = ok && i1 - i0 <= K;
    }
    return __syncthreads_and(ok) != 0;
}

// A table query resolved to its cell: the double2 offset of corner (ix, iy)
// at knot j, the bilinear weights and the spline abscissae.  Offsets are in
// range for any input (non-finite queries land in cell 0 or the last cell).
struct TabQ {
    uint32_t r;   // (row nd + j), row = ix ny + iy: the (F, M) table
    uint32_t rp;  // (row (nd - 1) + j): the FP32 knot-pair table (mixed precision)
    double tt, uu, d0, d1, dq;
};

__device__ __forceinline__ TabQ table_query(const TabArgs& t, const double* xs, const double* ys, const double* ds,
                                            const int* idx, double x, double y, double delta)
{
    const int ix = table_locate(t, 0, idx, xs, t.nx, x);
    const int iy = table_locate(t, 1, idx + t.nb[0], ys, t.ny, y);
    TabQ q;
    q.tt = fmin(fmax((x - xs[ix]) * rcp2(xs[ix + 1] - xs[ix]), 0.0), 1.0);
    q.uu = fmin(fmax((y - ys[iy]) * rcp2(ys[iy + 1] - ys[iy]), 0.0), 1.0);
    q.dq = fmin(fmax(delta, ds[0]), ds[t.nd - 1]);
    const int j = table_locate(t, 2, idx + t.nb[0] + t.nb[1], ds, t.nd, q.dq);
    q.d0 = ds[j];
    q.d1 = ds[j + 1];
    const int row = ix * t.ny + iy;
    q.r = (uint32_t)(row * t.nd + j);
    q.rp = (uint32_t)(row * (t.nd - 1) + j);
    return q;
}

// The 4 corners x 2 knots of a query's cell: c[2 * corner + {0, 1}], corners
// (ix, iy), (ix, iy + 1), (ix + 1, iy), (ix + 1, iy + 1).  (The table is
// passed as its own restrict-qualified pointer so that its reads are known
// not to alias the kernels' stores.)
__device__ __forceinline__ void table_load_from(const double* __restrict__ tab, const TabArgs& t, const TabQ& q,
                                               double2 (&c)[8])
{
    const double2* p = reinterpret_cast<const double2*>(tab) + q.r;
    const uint32_t sy = (uint32_t)t.nd;
    const uint32_t sx = (uint32_t)t.ny * sy;
    c[0] = p[0];
    c[1] = p[1];
    c[2] = p[sy];
    c[3] = p[sy + 1];
    c[4] = p[sx];
    c[5] = p[sx + 1];
    c[6] = p[sx + sy];
    c[7] = p[sx + sy + 1];
}

__device__ __forceinline__ void table_load(const TabArgs& t, const TabQ& q, double2 (&c)[8])
{
    table_load_from(t.tab, t, q, c);
}

// Splines in delta at the four corners, then bilinear; clamped to >= 0.
__device__ __forceinline__ double table_eval(const TabQ& q, const double2 (&c)[8])
{
    const double v00 = spline_piece(q.d0, q.d1, c[0].x, c[1].x, c[0].y, c[1].y, q.dq);
    const double v01 = spline_piece(q.d0, q.d1, c[2].x, c[3].x, c[2].y, c[3].y, q.dq);
    const double v10 = spline_piece(q.d0, q.d1, c[4].x, c[5].x, c[4].y, c[5].y, q.dq);
    const double v11 = spline_piece(q.d0, q.d1, c[6].x, c[7].x, c[6].y, c[7].y, q.dq);
    const double tt = q.tt, uu = q.uu;
    const double f = (1.0 - tt) * (1.0 - uu) * v00 + tt * (1.0 - uu) * v10 + (1.0 - tt) * uu * v01 + tt * uu * v11;
    return f > 0.0 ? f : 0.0;
}

// The table at (x, y, delta): splines in delta at the four corners of the
// (x, y) cell, then bilinear; knots xs, ys, ds and the index in LDS.  The
// same arithmetic as table_load + table_eval, but each corner is read and
// evaluated in turn: a kernel with one query per lane keeps half the
// registers live (42 against 84 VGPRs) and runs at higher occupancy.
__device__ __forceinline__ double table_corner(const double* __restrict__ tab, uint32_t o, const TabQ& q)
{
    const double2* p = reinterpret_cast<const double2*>(tab) + o;
    const double2 lo = p[0];
    const double2 hi = p[1];
    return spline_piece(q.d0, q.d1, lo.x, hi.x, lo.y, hi.y, q.dq);
}

__device__ __forceinline__ double table_at(const TabArgs& t, const double* xs, const double* ys, const double* ds,
                                           const int* idx, double x, double y, double delta)
{
    const TabQ q = table_query(t, xs, ys, ds, idx, x, y, delta);
    const uint32_t sy = (uint32_t)t.nd;
    const uint32_t sx = (uint32_t)t.ny * sy;
    const double v00 = table_corner(t.tab, q.r, q);
    const double v01 = table_corner(t.tab, q.r + sy, q);
    const double v10 = table_corner(t.tab, q.r + sx, q);
    const double v11 = table_corner(t.tab, q.r + sx + sy, q);
    const double tt = q.tt, uu = q.uu;
    const double f = (1.0 - tt) * (1.0 - uu) * v00 + tt * (1.0 - uu) * v10 + (1.0 - tt) * uu * v01 + tt * uu * v11;
    return f > 0.0 ? f : 0.0;
}

// Stage the scaled knots and the interval index at `base` (LDS); returns the
// index's LDS address.
__device__ __forceinline__ const int* stage_table(double* base, const TabArgs& t)
{
    double* xs = base;
    double* ys = xs + t.nx;
    double* ds = ys + t.ny;
    int* idx = reinterpret_cast<int*>(ds + t.nd);
    for (int k = threadIdx.x; k < t.nx; k += blockDim.x)
        xs[k] = t.xk[k] * t.scale;
    for (int k = threadIdx.x; k < t.ny; k += blockDim.x)
        ys[k] = t.yk[k] * t.scale;
    for (int k = threadIdx.x; k < t.nd; k += blockDim.x)
        ds[k] = t.dk[k] * t.scale;
    if (t.indexed)
        for (int k = threadIdx.x; k < t.nb[0] + t.nb[1] + t.nb[2]; k += blockDim.x)
            idx[k] = t.bidx[k];
    return idx;
}

// Eigenvalues of one particle and its table query (delta = l1 + l2 + l3,
// x = l1 - l2, y = l2 - l3); `finite` is false for non-finite eigenvalues,
// whose F is 0.
__device__ __forceinline__ TabQ tabulated_query(const TabArgs& t, const double* xs, const double* ys,
                                                const double* ds, const int* idx, const Hess64& h, bool& finite)
{
    double l1, l2, l3;
    eig_all(h, l1, l2, l3);
    finite = isfinite(l1) && isfinite(l2) && isfinite(l3);
    return table_query(t, xs, ys, ds, idx, l1 - l2, l2 - l3, l1 + l2 + l3);
}

__device__ __forceinline__ double tabulated_of(const TabArgs& t, const double* xs, const double* ys,
                                              const double* ds, const int* idx, const Hess64& h)
{
    bool finite;
    const TabQ q = tabulated_query(t, xs, ys, ds, idx, h, finite);
    double2 c[8];
    table_load(t, q, c);
    const double F = table_eval(q, c);
    return finite ? F : 0.0;
}

__global__ void __launch_bounds__(256) k_tabulated_f64_1(ItemArgs a, TabArgs t)
{
    extern __shared__ double lds[];
    double* g = lds;
    const GrowthIndex gi = stage_growth(lds, a);
    double* xs = lds + growth_lds_bytes(a.nk, a.gi.nb) / sizeof(double);
    double* ys = xs + t.nx;
    double* ds = ys + t.ny;
    const int* idx = stage_table(xs, t);
    __syncthreads();
    // One particle per lane (arrays not 16-byte aligned); the next element's
    // loads issued ahead of the current arithmetic.
    const uint32_t n = (uint32_t)a.n;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    Hess64 hn{};
    double fn = 0.0;
    if (i < n) {
        hn = load_h64(a, i);
        fn = a.reset ? 0.0 : *elem(a.Fmax, i);
    }
    for (; i < n; i += stride) {
        const Hess64 h = hn;
        const double fm = fn;
        const uint32_t next = i + stride;
        if (next < n) {
            hn = load_h64(a, next);
            fn = a.reset ? 0.0 : *elem(a.Fmax, next);
        }
        update_max(a, g, gi, i, tabulated_of(t, xs, ys, ds, idx, h), fm);
    }
}

// Two adjacent particles per lane, as k_classic_f64.  Both particles' cells
// are located before either's corners are read, so all 16 corner gathers of
// the lane are in flight together.
__global__ void __launch_bounds__(256) k_tabulated_f64(ItemArgs a, TabArgs t)
{
    extern __shared__ double lds[];
    double* g = lds;
    const GrowthIndex gi = stage_growth(lds, a);
    double* xs = lds + growth_lds_bytes(a.nk, a.gi.nb) / sizeof(double);
    double* ys = xs + t.nx;
    double* ds = ys + t.ny;
    const int* idx = stage_table(xs, t);
    __syncthreads();
    const uint32_t n = (uint32_t)a.n;
    const uint32_t np = n / 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    Hess2 hn{};
    d2v fn{0.0, 0.0};
    if (p < np) {
        hn = load_h2(a, p);
        if (!a.reset)
            fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * p));
    }
    for (; p < np; p += stride) {
        const Hess2 h = hn;
        const d2v fm = fn;
        const uint32_t next = p + stride;
        if (next < np) {
            hn = load_h2(a, next);
            if (!a.reset)
                fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * next));
        }
        bool f0, f1;
        const TabQ q0 = tabulated_query(t, xs, ys, ds, idx, Hess64{h.xx.x, h.yy.x, h.zz.x, h.xy.x, h.xz.x, h.yz.x}, f0);
        const TabQ q1 = tabulated_query(t, xs, ys, ds, idx, Hess64{h.xx.y, h.yy.y, h.zz.y, h.xy.y, h.xz.y, h.yz.y}, f1);
        double2 c0[8], c1[8];
        table_load(t, q0, c0);
        table_load(t, q1, c1);
        const double F0 = table_eval(q0, c0);
        const double F1 = table_eval(q1, c1);
        update_pair(a, g, gi, p, f0 ? F0 : 0.0, f1 ? F1 : 0.0, fm);
    }
    if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t i = n - 1;
        const double fm = a.reset ? 0.0 : *elem(a.Fmax, i);
        update_max(a, g, gi, i, tabulated_of(t, xs, ys, ds, idx, load_h64(a, i)), fm);
    }
}

// LDS bytes of stage_table
__host__ __device__ inline size_t table_lds_bytes(const TabArgs& t)
{
    return sizeof(double) * ((size_t)t.nx + t.ny + t.nd) +
           (t.indexed ? sizeof(int) * ((size_t)t.nb[0] + t.nb[1] + t.nb[2]) : 0);
}

// Interval index of a growth table (see GrowthIndex): bin b covers
// log2 D in [L0 + b/S, L0 + (b+1)/S), widened by a margin far above the FP32
// rounding of the lookup; idx[b] is the interval of the bin's low end and
// need[b] the number of compares the bin's high end needs beyond it.
__global__ void __launch_bounds__(256) k_growth_index(const double* __restrict__ D, int n, int nb, double L0,
                                                     double S, int* __restrict__ idx, int* __restrict__ need)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb)
        return;
    const double margin = 1e-4;
    const double lo = exp2(L0 + b / S - margin);
    const double hi = exp2(L0 + (b + 1) / S + margin);
    const int i0 = locate(D, n, lo);
    const int i1 = locate(D, n, hi);
    idx[b] = i0;
    need[b] = i1 - i0;
}

}  // namespace pino
