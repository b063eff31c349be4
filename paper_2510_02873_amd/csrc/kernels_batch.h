// Persistent batched kernel: a static list of particle tiles over many
// realisations, each particle carried through all of its radii with the
// running maximum in registers.
#pragma once

#include "kernels_fp64.h"
#include "kernels_mixed.h"

namespace pino {

struct RealDesc {
    int64_t n;
    int32_t n_radii;
    int32_t cosmo;
    int32_t radius_offset;
    int32_t nk;
    const void* const* h;  // device array, n_radii * 6 pointers, radius-major
    double* Fmax;
    int32_t* Rmax;
    double* acoll;
    const double* growth;  // [D | a | M] (FP64)
    const float* growth32; // FP32 copy (mixed precision), or null
    GrowthIndex gi;        // idx in global memory
    int32_t paired;        // arrays aligned for two particles per lane
};

template <bool F32> struct HessSel { using type = Hess64; using elem = double; };
template <> struct HessSel<true> { using type = Hess32; using elem = float; };
template <bool F32> using HessT = typename HessSel<F32>::type;

// Six streamed components of one particle; hp points at one radius' six
// component pointers.
template <bool F32>
__device__ __forceinline__ HessT<F32> load_hess(const void* const* hp, int64_t i)
{
    using E = typename HessSel<F32>::elem;
    HessT<F32> h;
    h.xx = __builtin_nontemporal_load(static_cast<const E*>(hp[0]) + i);
    h.yy = __builtin_nontemporal_load(static_cast<const E*>(hp[1]) + i);
    h.zz = __builtin_nontemporal_load(static_cast<const E*>(hp[2]) + i);
    h.xy = __builtin_nontemporal_load(static_cast<const E*>(hp[3]) + i);
    h.xz = __builtin_nontemporal_load(static_cast<const E*>(hp[4]) + i);
    h.yz = __builtin_nontemporal_load(static_cast<const E*>(hp[5]) + i);
    return h;
}

// F of one particle's Hessian at one radius (FP32 eigenvalues with the FP64
// fallback when F32, else FP64), then the FP64 root.
template <bool F32>
__device__ __forceinline__ double batch_F(const HessT<F32>& h)
{
    double l1, s, pp;
    if constexpr (F32) {
        float l1f, sf, ppf;
        if (eig_top_f32(h, l1f, sf, ppf)) {
            l1 = l1f;
            s = sf;
            pp = ppf;
        } else {
            eig_top(widen(h), l1, s, pp);
        }
    } else {
        eig_top(h, l1, s, pp);
    }
    return classic_F(l1, s, pp);
}

// The six components of particles i and i + 1 (i even, arrays aligned to two
// elements) at one radius, as two Hessians.
template <bool F32>
__device__ __forceinline__ void load_hess2(const void* const* hp, int64_t i, HessT<F32>& h0, HessT<F32>& h1)
{
    using E = typename HessSel<F32>::elem;
    typedef E V2 __attribute__((ext_vector_type(2)));
    V2 v[6];
    for (int c = 0; c < 6; ++c)
        v[c] = __builtin_nontemporal_load(reinterpret_cast<const V2*>(static_cast<const E*>(hp[c]) + i));
    h0 = HessT<F32>{v[0].x, v[1].x, v[2].x, v[3].x, v[4].x, v[5].x};
    h1 = HessT<F32>{v[0].y, v[1].y, v[2].y, v[3].y, v[4].y, v[5].y};
}

struct Tile {
    int32_t real;
    int32_t pad;
    int64_t start;
    int64_t count;
};

// One pass over the tiles assigned to this block (b, b + grid, ...).  The
// growth knots of a tile's cosmology are staged in LDS when the cosmology
// changes from the previous tile's.
template <bool F32>
__global__ void __launch_bounds__(256) k_batch(const RealDesc* __restrict__ reals, const Tile* __restrict__ tiles,
                                              int64_t n_tiles, uint32_t reset)
{
    extern __shared__ double lds[];
    int staged = -1;
    GrowthIndex gi{};
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const Tile tl = tiles[t];
        const RealDesc& R = reals[tl.real];
        const int nk = R.nk;
        if (R.cosmo != staged) {
            __syncthreads();
            if (F32) {
                float* g = reinterpret_cast<float*>(lds);
                for (int k = threadIdx.x; k < 3 * nk; k += blockDim.x)
                    g[k] = R.growth32[k];
                int* idx = reinterpret_cast<int*>(g + 3 * nk);
                for (int k = threadIdx.x; k < R.gi.nb; k += blockDim.x)
                    idx[k] = R.gi.idx[k];
                gi = R.gi;
                gi.idx = idx;
            } else {
                for (int k = threadIdx.x; k < 3 * nk; k += blockDim.x)
                    lds[k] = R.growth[k];
                int* idx = reinterpret_cast<int*>(lds + 3 * nk);
                for (int k = threadIdx.x; k < R.gi.nb; k += blockDim.x)
                    idx[k] = R.gi.idx[k];
                gi = R.gi;
                gi.idx = idx;
            }
            __syncthreads();
            staged = R.cosmo;
        }
        const int nr = R.n_radii;
        auto acoll_of = [&](double fm) {
            if (!(fm > 0.0))
                return kInf;
            if constexpr (F32)
                return (double)growth_invert_f32(reinterpret_cast<const float*>(lds), nk, (float)rcp2(fm), gi);
            else
                return growth_invert(lds, nk, rcp2(fm), gi);
        };
        // one particle through all radii: the next radius' Hessian is loaded
        // before the current one's arithmetic
        auto single = [&](int64_t i) {
            double fm = reset ? 0.0 : R.Fmax[i];
            int32_t rm = reset ? -1 : R.Rmax[i];
            HessT<F32> hn = load_hess<F32>(R.h, i);
            for (int r = 0; r < nr; ++r) {
                const HessT<F32> h = hn;
                if (r + 1 < nr)
                    hn = load_hess<F32>(R.h + 6 * (r + 1), i);
                const double F = batch_F<F32>(h);
                if (F > fm) {
                    fm = F;
                    rm = R.radius_offset + r;
                }
            }
            R.Fmax[i] = fm;
            R.Rmax[i] = rm;
            if (R.acoll)
                R.acoll[i] = acoll_of(fm);
        };
        if (R.paired) {
            // two adjacent particles per lane (tile starts are even): two
            // independent chains of eigen/root arithmetic per lane
            for (int64_t j = 2 * (int64_t)threadIdx.x; j < tl.count; j += 2 * (int64_t)blockDim.x) {
                const int64_t i = tl.start + j;
                if (j + 1 >= tl.count) {
                    single(i);
                    continue;
                }
                d2v fm{0.0, 0.0};
                int2 rm{-1, -1};
                if (!reset) {
                    fm = *reinterpret_cast<const d2v*>(R.Fmax + i);
                    rm = *reinterpret_cast<const int2*>(R.Rmax + i);
                }
                HessT<F32> n0, n1;
                load_hess2<F32>(R.h, i, n0, n1);
                for (int r = 0; r < nr; ++r) {
                    const HessT<F32> h0 = n0, h1 = n1;
                    if (r + 1 < nr)
                        load_hess2<F32>(R.h + 6 * (r + 1), i, n0, n1);
                    const double F0 = batch_F<F32>(h0);
                    const double F1 = batch_F<F32>(h1);
                    if (F0 > fm.x) {
                        fm.x = F0;
                        rm.x = R.radius_offset + r;
                    }
                    if (F1 > fm.y) {
                        fm.y = F1;
                        rm.y = R.radius_offset + r;
                    }
                }
                *reinterpret_cast<d2v*>(R.Fmax + i) = fm;
                *reinterpret_cast<int2*>(R.Rmax + i) = rm;
                if (R.acoll)
                    *reinterpret_cast<d2v*>(R.acoll + i) = d2v{acoll_of(fm.x), acoll_of(fm.y)};
            }
        } else {
            for (int64_t j = threadIdx.x; j < tl.count; j += blockDim.x)
                single(tl.start + j);
        }
    }
}

}  // namespace pino
