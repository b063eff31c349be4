// Surrogate + certify collapse kernel, network-input and prediction kernels.
#pragma once

#include "kernels_fp64.h"
#include "kernels_mixed.h"
#include "surrogate.h"

namespace pino {

// The Hessian of an item as FP64 (FP64 inputs) or widened FP32 inputs.
__device__ __forceinline__ Hess64 load_h(const ItemArgs& a, uint32_t i, bool f32)
{
    return f32 ? widen(load_h32(a, i)) : load_h64(a, i);
}

// LDS layout of k_surrogate: the growth knots and index (stage_growth), then
// the weight fragments at the next 16-byte boundary (they are copied and read
// as 16-byte vectors).
__host__ __device__ inline size_t net_lds_offset(int nk, int nb)
{
    return (growth_lds_bytes(nk, nb) + 15) / 16 * 16;
}

__host__ __device__ inline size_t surrogate_lds_bytes(int nk, int nb)
{
    return net_lds_offset(nk, nb) + sizeof(NetFrags);
}

// Per particle: FP64 eigenvalues of the FP64 Hessian, the BF16 network's
// prediction and the FP64 certificate.  The certificate brackets the first
// root of the particle's own cubic (built from its FP64 Hessian), so an
// accepted value is within rtol of the full solve on the same input.
// Certified and gated particles (F from the certificate, or 0) update the
// maxima in the main loop.  The others are deferred: each block appends their
// indices to its own segment of `queue` (queue + blockIdx.x * seg, seg >= the
// particles a block visits) through an LDS counter, one LDS atomic per wave,
// and carries their maxima over unchanged.  After its loop the block finishes
// its own deferred particles with the full FP64 Classic solve and updates
// their maxima against what the loop stored (at FINALIZE their a(D_c) is
// rewritten where F wins), so the full solve costs only the particles that
// need it, with no second launch.  The main loop is wave-uniform (all 64
// lanes run the network together); lanes past the end compute on zeros and
// store nothing.  counters: certified; consulted but not certified (full
// solve); not consulted with l1 > 0 (full solve); l1 <= 0 (F = 0, no solve).
// The waves of a block sum their counts in LDS and one lane adds the block's
// totals to the block's own four slots (counters + 4 blockIdx.x): a
// device-wide atomic on one shared address from every wave serialises at the
// coherence point and cost a few hundred microseconds per launch.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_surrogate(ItemArgs a, const NetFrags* __restrict__ net, double sigma,
                                                  double omega_m, double rtol,
                                                  unsigned long long* __restrict__ counters,
                                                  int32_t* __restrict__ queue, int64_t seg)
{
    extern __shared__ double lds[];
    __shared__ int fill;
    __shared__ unsigned long long bcount[4];
    const GrowthIndex gi = stage_growth(lds, a);
    NetFrags* N = reinterpret_cast<NetFrags*>(reinterpret_cast<char*>(lds) + net_lds_offset(a.nk, a.gi.nb));
    {
        const int4* src = reinterpret_cast<const int4*>(net);
        int4* dst = reinterpret_cast<int4*>(N);
        for (int k = threadIdx.x; k < (int)(sizeof(NetFrags) / sizeof(int4)); k += blockDim.x)
            dst[k] = src[k];
    }
    if (threadIdx.x == 0)
        fill = 0;
    if (threadIdx.x < 4)
        bcount[threadIdx.x] = 0;
    __syncthreads();
    int32_t* myq = queue + (int64_t)blockIdx.x * seg;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long ncert = 0, nfall = 0, ngsolve = 0, ngzero = 0;
    // the next group's Hessian loads are issued before the current group's
    // network and certificate (3 % faster).  The weight fragments stay in
    // registers across the loop (96 VGPRs; reading them from LDS in every
    // pass cost 3.5x), which leaves room for the six components only: Fmax
    // is read where it is used.
    int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    Hess64 hn{};
    if (base + lane < a.n)
        hn = load_h64(a, (uint32_t)(base + lane));
    for (; base < a.n; base += stride) {
        const bool valid = base + lane < a.n;
        const uint32_t i = (uint32_t)(base + lane);
        const Hess64 h = hn;
        if (base + stride + lane < a.n)
            hn = load_h64(a, (uint32_t)(base + stride + lane));
        const double fm = valid && !a.reset ? *elem(a.Fmax, i) : 0.0;
        double l1, s, pp;
        eig_top(h, l1, s, pp);
        float x[4];
        const bool consult = net_inputs(l1, s, pp, sigma, omega_m, x) && valid;
        if (!consult)
            x[0] = x[1] = x[2] = x[3] = 0.0f;
        const float y = net_bf16(*N, x);
        double F = 0.0;
        bool cert = false;
        if (l1 > 0.0) {
            const CubicU k = lpt_cubic(l1, s, pp, rcp2(l1));
            double u1;
            if (consult && certify(k, (double)y, rtol, u1)) {
                F = l1 * rcp2(u1);
                cert = true;
            }
        }
        // l1 > 0 and not certified: deferred to the full solve
        const bool defer = valid && l1 > 0.0 && !cert;
        const uint64_t dm = __ballot(defer);
        if (dm) {
            int slot = 0;
            if (lane == 0)
                slot = atomicAdd(&fill, (int)__popcll(dm));
            slot = __shfl(slot, 0, 64);
            if (defer)
                myq[slot + (int)__popcll(dm & below)] = (int32_t)i;
        }
        ncert += __popcll(__ballot(valid && cert));
        nfall += __popcll(__ballot(consult && !cert));
        ngsolve += __popcll(__ballot(valid && !consult && l1 > 0.0));
        ngzero += __popcll(__ballot(valid && !(l1 > 0.0)));
        if (valid)
            update_max(a, lds, gi, i, F, fm);
    }
    if (lane == 0) {
        atomicAdd(&bcount[0], ncert);
        atomicAdd(&bcount[1], nfall);
        atomicAdd(&bcount[2], ngsolve);
        atomicAdd(&bcount[3], ngzero);
    }
    // the block's queue entries and the maxima its loop stored are visible
    // to the whole block after the barrier
    __syncthreads();
    if (threadIdx.x < 4 && counters)
        atomicAdd(counters + 4 * (int64_t)blockIdx.x + threadIdx.x, bcount[threadIdx.x]);
    const int count = fill;
    for (int qi = threadIdx.x; qi < count; qi += blockDim.x) {
        const uint32_t i = (uint32_t)myq[qi];
        double l1, s, pp;
        eig_top(load_h64(a, i), l1, s, pp);
        const double F = classic_F(l1, s, pp);
        if (F > *elem(a.Fmax, i)) {
            *elem(a.Fmax, i) = F;
            *elem(a.Rmax, i) = a.radius;
            if (a.acoll)
                *elem(a.acoll, i) = growth_invert(lds, a.nk, rcp2(F), gi);
        }
    }
}

// Network inputs x [n][4] and target w = 1/(l1 D_c) (0 where the network is
// not consulted) from the full FP64 solve.
__global__ void __launch_bounds__(256) k_features(ItemArgs a, bool f32, double sigma, double omega_m,
                                                 float* __restrict__ X, float* __restrict__ W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    const Hess64 h = load_h(a, (uint32_t)i, f32);
    double l1, s, pp;
    eig_top(h, l1, s, pp);
    float x[4];
    const bool consult = net_inputs(l1, s, pp, sigma, omega_m, x);
    for (int k = 0; k < 4; ++k)
        X[i * 4 + k] = x[k];
    if (W) {
        const double F = consult ? classic_F(l1, s, pp) : 0.0;
        W[i] = F > 0.0 ? (float)(F / l1) : 0.0f;
    }
}

// The BF16 network on given inputs (wave-uniform loop)
__global__ void __launch_bounds__(256) k_predict(const NetFrags* __restrict__ net, const float* __restrict__ X,
                                                float* __restrict__ Y, int64_t n)
{
    __shared__ NetFrags N;
    {
        const int4* src = reinterpret_cast<const int4*>(net);
        int4* dst = reinterpret_cast<int4*>(&N);
        for (int k = threadIdx.x; k < (int)(sizeof(NetFrags) / sizeof(int4)); k += blockDim.x)
            dst[k] = src[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t i = base + lane;
        float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (i < n)
            for (int k = 0; k < 4; ++k)
                x[k] = X[i * 4 + k];
        const float y = net_bf16(N, x);
        if (i < n)
            Y[i] = y;
    }
}

}  // namespace pino
