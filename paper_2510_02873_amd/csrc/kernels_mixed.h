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

}  // namespace pino
