// Surrogate + certify collapse kernel, network-input and prediction kernels.
#pragma once

#include "kernels_fp64.h"
#include "kernels_lcdm.h"
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
// as 16-byte vectors), then for the LCDM method the six ratio rows of the
// item's cosmology (nk doubles each).
__host__ __device__ inline size_t net_lds_offset(int nk, int nb)
{
    return (growth_lds_bytes(nk, nb) + 15) / 16 * 16;
}

__host__ __device__ inline size_t surrogate_lds_bytes(int nk, int nb, bool lcdm = false)
{
    return net_lds_offset(nk, nb) + sizeof(NetFrags) + (lcdm ? 6 * (size_t)nk * sizeof(double) : 0);
}

// ---------------------------------------------------------------------------
// Certificate of the LCDM method.  G(u) = 1 - u + k2(D) b u^2 +
// (k3a(D) ca + k3b(D) cb) u^3 with D = u / l1 is a cubic whose coefficients
// move slowly with D.  From the prediction u0 = 1/y, one Newton step on G
// (ratio derivatives included) gives u1; it is accepted as G's first root
// within rtol when
//   (i)  G(lo) > e and G(hi) < -e at lo, hi = u1 (1 -/+ rtol), e four times
//        the Horner bound of g_bound (the ratios' own rounding is below it);
//   (ii) G > 0 on (0, lo].  With F the cubic whose ratios are frozen at their
//        values at D_lo = lo / l1, and K_j bounds on |d k_j / d ln D| over the
//        whole table (kslope, computed at init), |k_j(D) - k_j(D_lo)| <=
//        K_j ln(lo/u) <= K_j (lo - u)/u for u <= lo, so
//        |G(u) - F(u)| <= es (lo - u), es = K2 |b| lo + (K3a |ca| + K3b |cb|) lo^2,
//        and G >= Ft = F - es (lo - u), itself a cubic with Ft(0) = 1 - es lo,
//        Ft'(0) = -(1 - es) and Ft(lo) = G(lo) > 0.  Ft > 0 on (0, lo] then
//        follows from the same critical-point test as the Einstein-de Sitter
//        certificate: its first positive critical point um (a minimum, since
//        Ft'(0) < 0) lies at or past lo, or Ft(um) > e.
// ---------------------------------------------------------------------------
struct KappaSlope {
    double k2, k3a, k3b;
};

// G at u with a fresh lookup of the ratios (the spline piece is not kept in
// registers across the certificate: beside the network's weights it spilled)
__device__ __forceinline__ double lcdm_G(double u, double il1, double b, double ca, double cb, const double* g,
                                         const double* kap, int nk, const GrowthIndex& gi, double& P, double& Q)
{
    const double D = u * il1;
    const Kappa k = kappa_eval(kappa_piece(g, kap, nk, D, gi), D);
    P = k.k2 * b;
    Q = k.k3a * ca + k.k3b * cb;
    return 1.0 + u * (-1.0 + u * (P + Q * u));
}

__device__ __forceinline__ bool certify_lcdm(double l1, double il1, double b, double ca, double cb, double y,
                                             double rtol, const KappaSlope& ks, const double* g, const double* kap,
                                             int nk, const GrowthIndex& gi, double& u1)
{
    if (!(y > 0.0) || !isfinite(y))
        return false;
    const double u0 = rcp2(y);
    const double D0 = u0 * il1;
    const Kappa k = kappa_eval(kappa_piece(g, kap, nk, D0, gi), D0);
    const double P0 = k.k2 * b;
    const double Q0 = k.k3a * ca + k.k3b * cb;
    const double G0 = 1.0 + u0 * (-1.0 + u0 * (P0 + Q0 * u0));
    const double dG0 = -1.0 + u0 * (2.0 * P0 + 3.0 * Q0 * u0) +
                       (u0 * u0) * il1 * (k.d2 * b + u0 * (k.d3a * ca + k.d3b * cb));
    u1 = u0 - G0 * rcp2(dG0);
    const double lo = u1 * (1.0 - rtol);
    const double hi = u1 * (1.0 + rtol);
    if (!(lo > 0.0) || !isfinite(u1))
        return false;
    double Pl, Ql, Ph, Qh;
    const double Glo = lcdm_G(lo, il1, b, ca, cb, g, kap, nk, gi, Pl, Ql);
    const double Ghi = lcdm_G(hi, il1, b, ca, cb, g, kap, nk, gi, Ph, Qh);
    const bool bracket = Glo > 4.0 * g_bound(CubicU{Pl, Ql}, lo) && Ghi < -4.0 * g_bound(CubicU{Ph, Qh}, hi);
    const double es = ks.k2 * fabs(b) * lo + (ks.k3a * fabs(ca) + ks.k3b * fabs(cb)) * (lo * lo);
    if (!(es * lo < 1.0) || !(es < 1.0))
        return false;
    // Ft(u) = c0 + c1 u + Pl u^2 + Ql u^3
    const double c0 = 1.0 - es * lo;
    const double c1 = -(1.0 - es);
    const double disc = Pl * Pl - 3.0 * Ql * c1;
    const double den = Pl + sqrt(fmax(disc, 0.0));
    bool earlier = false;
    if (disc >= 0.0 && den > 0.0) {
        const double um = -c1 * rcp2(den);
        if (um < lo) {
            const double Fm = c0 + um * (c1 + um * (Pl + Ql * um));
            earlier = !(Fm > 4.0 * g_bound(CubicU{Pl, Ql}, um));
        }
    }
    return bracket && !earlier;
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
// LCDM: the same with the LCDM condition (certify_lcdm, the full solve of
// lcdm_F); kap_all: the item's ratio rows, ks: their slope bounds.
template <bool LCDM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_surrogate(ItemArgs a, const NetFrags* __restrict__ net, double sigma,
                                                  double omega_m, double rtol,
                                                  unsigned long long* __restrict__ counters,
                                                  int32_t* __restrict__ queue, int64_t seg,
                                                  const double* __restrict__ kap_all, KappaSlope ks)
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
    double* kap = reinterpret_cast<double*>(N + 1);
    if constexpr (LCDM)
        stage(kap, kap_all, 6 * a.nk);
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
            const double il1 = rcp2(l1);
            double u1;
            bool ok;
            if constexpr (LCDM) {
                const double sg = s * il1;
                const double pi = pp * (il1 * il1);
                const double b = (-3.0 / 14.0) * sg;
                const double ca = pi * (1.0 / 9.0);
                const double cb = -(sg * (1.0 / 56.0) + pi * (2.0 / 56.0) + (17.0 / 168.0) * (sg * sg));
                ok = consult && certify_lcdm(l1, il1, b, ca, cb, (double)y, rtol, ks, lds, kap, a.nk, gi, u1);
            } else {
                ok = consult && certify(lpt_cubic(l1, s, pp, il1), (double)y, rtol, u1);
            }
            if (ok) {
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
        double F;
        if constexpr (LCDM)
            F = lcdm_F(l1, s, pp, KapRows{lds, kap, (int)a.nk, gi});
        else
            F = classic_F(l1, s, pp);
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
// kap: the LCDM ratio rows of the item's cosmology (global memory; NULL:
// the Einstein-de Sitter condition), with a.growth and a.gi for their knots.
__global__ void __launch_bounds__(256) k_features(ItemArgs a, bool f32, double sigma, double omega_m,
                                                 const double* __restrict__ kap, float* __restrict__ X,
                                                 float* __restrict__ W)
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
        double F = 0.0;
        if (consult)
            F = kap ? lcdm_F(l1, s, pp, KapRows{a.growth, kap, (int)a.nk, a.gi}) : classic_F(l1, s, pp);
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
