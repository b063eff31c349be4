// Mixed-precision Classic kernel: FP32 Hessians (24 B per particle), FP32
// eigenvalues with an FP64 branch for nearly repeated l1 ~ l2, the FP64
// collapse root (FP32 estimate + FP64 Halley polish), and a(D) interpolated
// in FP32 from FP32 copies of the growth knots.
#pragma once

#include "device_mixed.h"
#include "kernels_fp64.h"

namespace pino {

__device__ __forceinline__ Hess32 load_h32(const ItemArgs& a, uint32_t i)
{
    Hess32 h;
    h.xx = __builtin_nontemporal_load(elem(reinterpret_cast<const float*>(a.h[0]), i));
    h.yy = __builtin_nontemporal_load(elem(reinterpret_cast<const float*>(a.h[1]), i));
    h.zz = __builtin_nontemporal_load(elem(reinterpret_cast<const float*>(a.h[2]), i));
    h.xy = __builtin_nontemporal_load(elem(reinterpret_cast<const float*>(a.h[3]), i));
    h.xz = __builtin_nontemporal_load(elem(reinterpret_cast<const float*>(a.h[4]), i));
    h.yz = __builtin_nontemporal_load(elem(reinterpret_cast<const float*>(a.h[5]), i));
    return h;
}

// FP32 growth knots and the interval index into LDS
__device__ __forceinline__ GrowthIndex stage_growth32(float* lds, const float* __restrict__ g32, const ItemArgs& a)
{
    for (int k = threadIdx.x; k < 3 * a.nk; k += blockDim.x)
        lds[k] = g32[k];
    int* idx = reinterpret_cast<int*>(lds + 3 * a.nk);
    for (int k = threadIdx.x; k < a.gi.nb; k += blockDim.x)
        idx[k] = a.gi.idx[k];
    GrowthIndex gi = a.gi;
    gi.idx = idx;
    return gi;
}

// same whole-line update as update_max, with a(D) in FP32
__device__ __forceinline__ void update_max_f32(const ItemArgs& a, const float* g, const GrowthIndex& gi, uint32_t i,
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
            *ac = fnew > 0.0 ? (double)growth_invert_f32(g, a.nk, (float)rcp2(fnew), gi) : kInf;
        } else {
            const double am = a.reset ? kInf : *ac;
            *ac = upd ? (double)growth_invert_f32(g, a.nk, (float)rcp2(F), gi) : am;
        }
    }
}

__global__ void __launch_bounds__(256) k_classic_mixed_1(ItemArgs a, const float* __restrict__ growth32)
{
    extern __shared__ double lds[];
    float* g = reinterpret_cast<float*>(lds);
    const GrowthIndex gi = stage_growth32(g, growth32, a);
    __syncthreads();
    // One particle per lane (arrays not 8/16-byte aligned); the next
    // element's loads issued ahead of the current arithmetic.
    const uint32_t n = (uint32_t)a.n;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    Hess32 hn{};
    double fn = 0.0;
    if (i < n) {
        hn = load_h32(a, i);
        fn = a.reset ? 0.0 : *elem(a.Fmax, i);
    }
    for (; i < n; i += stride) {
        const Hess32 h = hn;
        const double fm = fn;
        const uint32_t next = i + stride;
        if (next < n) {
            hn = load_h32(a, next);
            fn = a.reset ? 0.0 : *elem(a.Fmax, next);
        }
        float l1f, sf, ppf;
        double l1, s, pp;
        if (eig_top_f32(h, l1f, sf, ppf)) {
            l1 = l1f;
            s = sf;
            pp = ppf;
        } else {
            eig_top(widen(h), l1, s, pp);
        }
        const double F = classic_F(l1, s, pp);
        update_max_f32(a, g, gi, i, F, fm);
    }
}

// F of one particle from its FP32 Hessian: FP32 eigenvalues, or FP64 ones
// where the FP32 closed form is not trusted; FP64 root.
__device__ __forceinline__ double mixed_F(const Hess32& h)
{
    float l1f, sf, ppf;
    double l1, s, pp;
    if (eig_top_f32(h, l1f, sf, ppf)) {
        l1 = l1f;
        s = sf;
        pp = ppf;
    } else {
        eig_top(widen(h), l1, s, pp);
    }
    return classic_F(l1, s, pp);
}

typedef float f2v __attribute__((ext_vector_type(2)));

// update_max_f32 for the pair (2p, 2p + 1): 16-byte Fmax and a_coll, 8-byte
// Rmax accesses
__device__ __forceinline__ void update_pair_f32(const ItemArgs& a, const float* g, const GrowthIndex& gi, uint32_t p,
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
            v.x = fnew.x > 0.0 ? (double)growth_invert_f32(g, a.nk, (float)rcp2(fnew.x), gi) : kInf;
            v.y = fnew.y > 0.0 ? (double)growth_invert_f32(g, a.nk, (float)rcp2(fnew.y), gi) : kInf;
        } else {
            const d2v am = a.reset ? d2v{kInf, kInf} : *ac;
            v.x = u0 ? (double)growth_invert_f32(g, a.nk, (float)rcp2(F0), gi) : am.x;
            v.y = u1 ? (double)growth_invert_f32(g, a.nk, (float)rcp2(F1), gi) : am.y;
        }
        *ac = v;
    }
}

// Two adjacent particles per lane (8-byte component loads, 16-byte Fmax and
// a_coll, 8-byte Rmax; alignment checked by the host), as k_classic_f64.
__global__ void __launch_bounds__(256) k_classic_mixed(ItemArgs a, const float* __restrict__ growth32)
{
    extern __shared__ double lds[];
    float* g = reinterpret_cast<float*>(lds);
    const GrowthIndex gi = stage_growth32(g, growth32, a);
    __syncthreads();
    const uint32_t n = (uint32_t)a.n;
    const uint32_t np = n / 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    f2v hn[6];
    d2v fn{0.0, 0.0};
    auto load = [&](uint32_t q) {
        for (int c = 0; c < 6; ++c)
            hn[c] = __builtin_nontemporal_load(
                reinterpret_cast<const f2v*>(elem(reinterpret_cast<const float*>(a.h[c]), 2 * q)));
        if (!a.reset)
            fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * q));
    };
    if (p < np)
        load(p);
    for (; p < np; p += stride) {
        f2v h[6];
        for (int c = 0; c < 6; ++c)
            h[c] = hn[c];
        const d2v fm = fn;
        if (p + stride < np)
            load(p + stride);
        const double F0 = mixed_F(Hess32{h[0].x, h[1].x, h[2].x, h[3].x, h[4].x, h[5].x});
        const double F1 = mixed_F(Hess32{h[0].y, h[1].y, h[2].y, h[3].y, h[4].y, h[5].y});
        update_pair_f32(a, g, gi, p, F0, F1, fm);
    }
    if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t i = n - 1;
        const double fm = a.reset ? 0.0 : *elem(a.Fmax, i);
        update_max_f32(a, g, gi, i, mixed_F(load_h32(a, i)), fm);
    }
}

// FP32 copy of count doubles
__global__ void __launch_bounds__(256) k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        dst[i] = (float)src[i];
}

// LDS bytes of stage_growth32
__host__ __device__ inline size_t growth32_lds_bytes(int nk, int nb)
{
    return (((size_t)3 * nk * sizeof(float) + 7) / 8) * 8 + (((size_t)nb * sizeof(int) + 7) / 8) * 8;
}

// ---------------------------------------------------------------------------
// Mixed-precision Tabulated kernels: FP32 Hessians (24 B per particle), FP32
// eigenvalues (the FP64 path for nearly repeated pairs), the cell search in
// FP32 copies of the scaled knots, and FP32 interpolation on an FP32 copy of
// the table in which each (row, knot interval j) holds the 16-byte tuple
// (F_j, M_j, F_{j+1}, M_{j+1}), so one corner spline is one 16-byte read
// (four per particle instead of eight); a(D) from the FP32 growth knots, as
// in the mixed Classic kernel.
// ---------------------------------------------------------------------------

// tab32[r (nd - 1) + j] = (F_j, M_j, F_{j+1}, M_{j+1}) of row r, from the
// interleaved FP64 (F, M) table of the same radius
__global__ void __launch_bounds__(256) k_table_pairs_f32(const double* __restrict__ tab, f4v* __restrict__ tab32,
                                                        int rows, int nd)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)rows * (nd - 1))
        return;
    const int64_t r = k / (nd - 1);
    const int64_t j = k - r * (nd - 1);
    const double* s = tab + (r * nd + j) * 2;
    tab32[k] = f4v{(float)s[0], (float)s[1], (float)s[2], (float)s[3]};
}

// FP32 copies of the scaled knots [x | y | delta], then the interval index
// (at most table_lds_bytes(t) bytes)
__device__ __forceinline__ const int* stage_table32(float* base, const TabArgs& t)
{
    float* xs = base;
    float* ys = xs + t.nx;
    float* ds = ys + t.ny;
    int* idx = reinterpret_cast<int*>(ds + t.nd);
    for (int k = threadIdx.x; k < t.nx; k += blockDim.x)
        xs[k] = (float)(t.xk[k] * t.scale);
    for (int k = threadIdx.x; k < t.ny; k += blockDim.x)
        ys[k] = (float)(t.yk[k] * t.scale);
    for (int k = threadIdx.x; k < t.nd; k += blockDim.x)
        ds[k] = (float)(t.dk[k] * t.scale);
    if (t.indexed)
        for (int k = threadIdx.x; k < t.nb[0] + t.nb[1] + t.nb[2]; k += blockDim.x)
            idx[k] = t.bidx[k];
    return idx;
}

// locate_after and table_locate on FP32 knots.  The index bins carry a margin
// of 1 % of a bin, far above the FP32 rounding of the bin arithmetic and of
// the knots, so the bin's interval is never past the query's.
__device__ __forceinline__ int locate_after32(const float* xs, int n, float q, int i)
{
    constexpr int K = kIndexCompares;
    float xv[K];
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

__device__ __forceinline__ int table_locate32(const TabArgs& t, int axis, const int* idx, const float* xs, int n,
                                              float q)
{
    if (!t.indexed)
        return locate32(xs, n, q);
    float fb = (q * (float)t.inv_scale - (float)t.k0[axis]) * (float)t.bpu[axis];
    fb = fminf(fmaxf(fb, 0.0f), (float)(t.nb[axis] - 1));
    return locate_after32(xs, n, q, idx[(int)fb]);
}

struct TabQ32 {
    uint32_t rp;  // (row (nd - 1) + j) in the knot-pair table
    float tt, uu, d0, d1, dq;
};

__device__ __forceinline__ TabQ32 table_query32(const TabArgs& t, const float* xs, const float* ys, const float* ds,
                                                const int* idx, float x, float y, float delta)
{
    const int ix = table_locate32(t, 0, idx, xs, t.nx, x);
    const int iy = table_locate32(t, 1, idx + t.nb[0], ys, t.ny, y);
    TabQ32 q;
    q.tt = fminf(fmaxf((x - xs[ix]) / (xs[ix + 1] - xs[ix]), 0.0f), 1.0f);
    q.uu = fminf(fmaxf((y - ys[iy]) / (ys[iy + 1] - ys[iy]), 0.0f), 1.0f);
    q.dq = fminf(fmaxf(delta, ds[0]), ds[t.nd - 1]);
    const int j = table_locate32(t, 2, idx + t.nb[0] + t.nb[1], ds, t.nd, q.dq);
    q.d0 = ds[j];
    q.d1 = ds[j + 1];
    q.rp = (uint32_t)((ix * t.ny + iy) * (t.nd - 1) + j);
    return q;
}

// The cell of a particle from its FP32 Hessian: x = l1 - l2, y = l2 - l3 from
// the FP32 eigenvalues (FP64 for nearly repeated pairs, rounded to FP32
// after the differences), delta = the FP32 trace.
__device__ __forceinline__ TabQ32 tabulated_query32(const TabArgs& t, const float* xs, const float* ys,
                                                    const float* ds, const int* idx, const Hess32& h, bool& finite)
{
    float l1, l2, l3, x, y;
    if (eig_all_f32(h, l1, l2, l3)) {
        x = l1 - l2;
        y = l2 - l3;
    } else {
        double e1, e2, e3;
        eig_all(widen(h), e1, e2, e3);
        l1 = (float)e1;
        x = (float)(e1 - e2);
        y = (float)(e2 - e3);
    }
    const float delta = h.xx + h.yy + h.zz;
    finite = isfinite(x) && isfinite(y) && isfinite(delta) && isfinite(l1);
    return table_query32(t, xs, ys, ds, idx, x, y, delta);
}

// corners (ix, iy), (ix, iy + 1), (ix + 1, iy), (ix + 1, iy + 1)
__device__ __forceinline__ void table_load32(const TabArgs& t, const f4v* __restrict__ tab32, const TabQ32& q,
                                             f4v (&c)[4])
{
    const f4v* p = tab32 + q.rp;
    const uint32_t sy = (uint32_t)t.nd - 1;
    const uint32_t sx = (uint32_t)t.ny * sy;
    c[0] = p[0];
    c[1] = p[sy];
    c[2] = p[sx];
    c[3] = p[sx + sy];
}

__device__ __forceinline__ float table_eval32(const TabQ32& q, const f4v (&c)[4])
{
    const float v00 = spline_piece32(q.d0, q.d1, c[0].x, c[0].z, c[0].y, c[0].w, q.dq);
    const float v01 = spline_piece32(q.d0, q.d1, c[1].x, c[1].z, c[1].y, c[1].w, q.dq);
    const float v10 = spline_piece32(q.d0, q.d1, c[2].x, c[2].z, c[2].y, c[2].w, q.dq);
    const float v11 = spline_piece32(q.d0, q.d1, c[3].x, c[3].z, c[3].y, c[3].w, q.dq);
    const float tt = q.tt, uu = q.uu;
    const float f = (1.0f - tt) * (1.0f - uu) * v00 + tt * (1.0f - uu) * v10 + (1.0f - tt) * uu * v01 + tt * uu * v11;
    return f > 0.0f ? f : 0.0f;
}

__device__ __forceinline__ double tabulated_mixed_of(const TabArgs& t, const f4v* __restrict__ tab32,
                                                    const float* xs, const float* ys, const float* ds,
                                                    const int* idx, const Hess32& h)
{
    bool finite;
    const TabQ32 q = tabulated_query32(t, xs, ys, ds, idx, h, finite);
    f4v c[4];
    table_load32(t, tab32, q, c);
    const float F = table_eval32(q, c);
    return finite ? (double)F : 0.0;
}

// One particle per lane (FP32 components not 8-byte aligned).
__global__ void __launch_bounds__(256) k_tabulated_mixed_1(ItemArgs a, TabArgs t, const f4v* __restrict__ tab32,
                                                          const float* __restrict__ growth32)
{
    extern __shared__ double lds[];
    float* g = reinterpret_cast<float*>(lds);
    const GrowthIndex gi = stage_growth32(g, growth32, a);
    float* xs = g + growth32_lds_bytes(a.nk, a.gi.nb) / sizeof(float);
    float* ys = xs + t.nx;
    float* ds = ys + t.ny;
    const int* idx = stage_table32(xs, t);
    __syncthreads();
    const uint32_t n = (uint32_t)a.n;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    Hess32 hn{};
    double fn = 0.0;
    if (i < n) {
        hn = load_h32(a, i);
        fn = a.reset ? 0.0 : *elem(a.Fmax, i);
    }
    for (; i < n; i += stride) {
        const Hess32 h = hn;
        const double fm = fn;
        const uint32_t next = i + stride;
        if (next < n) {
            hn = load_h32(a, next);
            fn = a.reset ? 0.0 : *elem(a.Fmax, next);
        }
        update_max_f32(a, g, gi, i, tabulated_mixed_of(t, tab32, xs, ys, ds, idx, h), fm);
    }
}

// Two adjacent particles per lane (alignment as k_classic_mixed); both cells
// are located before the eight corner reads are issued.
__global__ void __launch_bounds__(256) k_tabulated_mixed(ItemArgs a, TabArgs t, const f4v* __restrict__ tab32,
                                                        const float* __restrict__ growth32)
{
    extern __shared__ double lds[];
    float* g = reinterpret_cast<float*>(lds);
    const GrowthIndex gi = stage_growth32(g, growth32, a);
    float* xs = g + growth32_lds_bytes(a.nk, a.gi.nb) / sizeof(float);
    float* ys = xs + t.nx;
    float* ds = ys + t.ny;
    const int* idx = stage_table32(xs, t);
    __syncthreads();
    const uint32_t n = (uint32_t)a.n;
    const uint32_t np = n / 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    f2v hn[6];
    d2v fn{0.0, 0.0};
    auto load = [&](uint32_t q) {
        for (int c = 0; c < 6; ++c)
            hn[c] = __builtin_nontemporal_load(
                reinterpret_cast<const f2v*>(elem(reinterpret_cast<const float*>(a.h[c]), 2 * q)));
        if (!a.reset)
            fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * q));
    };
    if (p < np)
        load(p);
    for (; p < np; p += stride) {
        f2v h[6];
        for (int c = 0; c < 6; ++c)
            h[c] = hn[c];
        const d2v fm = fn;
        if (p + stride < np)
            load(p + stride);
        bool f0, f1;
        const TabQ32 q0 =
            tabulated_query32(t, xs, ys, ds, idx, Hess32{h[0].x, h[1].x, h[2].x, h[3].x, h[4].x, h[5].x}, f0);
        const TabQ32 q1 =
            tabulated_query32(t, xs, ys, ds, idx, Hess32{h[0].y, h[1].y, h[2].y, h[3].y, h[4].y, h[5].y}, f1);
        f4v c0[4], c1[4];
        table_load32(t, tab32, q0, c0);
        table_load32(t, tab32, q1, c1);
        const float F0 = table_eval32(q0, c0);
        const float F1 = table_eval32(q1, c1);
        update_pair_f32(a, g, gi, p, f0 ? (double)F0 : 0.0, f1 ? (double)F1 : 0.0, fm);
    }
    if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t i = n - 1;
        const double fm = a.reset ? 0.0 : *elem(a.Fmax, i);
        update_max_f32(a, g, gi, i, tabulated_mixed_of(t, tab32, xs, ys, ds, idx, load_h32(a, i)), fm);
    }
}


}  // namespace pino
