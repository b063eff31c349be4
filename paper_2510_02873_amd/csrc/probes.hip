// Ceiling probes of the measurement harness: what the chip sustains for the
// access pattern and the arithmetic of the collapse kernels, measured on the
// box next to them (the spec sheet's 8 TB/s and 78.6 TFLOP/s are upper bounds
// that no kernel reaches).  Built as libpino_probes.so, separate from the
// collapse library; only the benchmark loads it.
//
//   pino_probe_copy       : a streaming copy, 16 bytes per lane per access,
//                           four accesses in flight per lane.
//   pino_probe_stream     : the data movement of the per-radius FP64 kernel
//                           with no arithmetic: six FP64 Hessian streams read
//                           with the nontemporal hint, the running maxima
//                           Fmax (f64) and Rmax (i32) read and written back as
//                           whole lines through the caches, pairs of
//                           particles per lane.  Its update is a plain
//                           comparison against the sum of the six components.
//   pino_probe_fma_f64    : independent FP64 fused multiply-add chains.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef int i4v __attribute__((ext_vector_type(4)));

// four coalesced 16-byte loads in flight per lane, then their stores
__global__ void __launch_bounds__(256) k_probe_copy(const i4v* __restrict__ src, i4v* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const i4v a = __builtin_nontemporal_load(src + i);
        const i4v b = __builtin_nontemporal_load(src + i + stride);
        const i4v c = __builtin_nontemporal_load(src + i + 2 * stride);
        const i4v d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void __launch_bounds__(256) k_probe_stream(const d2v* __restrict__ h0, const d2v* __restrict__ h1,
                                                     const d2v* __restrict__ h2, const d2v* __restrict__ h3,
                                                     const d2v* __restrict__ h4, const d2v* __restrict__ h5,
                                                     d2v* __restrict__ Fmax, int2* __restrict__ Rmax, int64_t np,
                                                     int radius)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        const d2v s = __builtin_nontemporal_load(h0 + p) + __builtin_nontemporal_load(h1 + p) +
                      __builtin_nontemporal_load(h2 + p) + __builtin_nontemporal_load(h3 + p) +
                      __builtin_nontemporal_load(h4 + p) + __builtin_nontemporal_load(h5 + p);
        const d2v fm = Fmax[p];
        const int2 rm = Rmax[p];
        const bool u0 = s.x > fm.x, u1 = s.y > fm.y;
        Fmax[p] = d2v{u0 ? s.x : fm.x, u1 ? s.y : fm.y};
        Rmax[p] = int2{u0 ? radius : rm.x, u1 ? radius : rm.y};
    }
}

// 8 independent chains per lane of iters FMAs each; out keeps them live
__global__ void __launch_bounds__(256) k_probe_fma_f64(double* __restrict__ out, int iters, double b)
{
    const double seed = 1.0 + 1e-9 * (blockIdx.x * blockDim.x + threadIdx.x);
    double c0 = seed, c1 = seed + 1e-3, c2 = seed + 2e-3, c3 = seed + 3e-3;
    double c4 = seed + 4e-3, c5 = seed + 5e-3, c6 = seed + 6e-3, c7 = seed + 7e-3;
    const double m = 0.999999999;
#pragma unroll 4
    for (int k = 0; k < iters; ++k) {
        c0 = fma(c0, m, b);
        c1 = fma(c1, m, b);
        c2 = fma(c2, m, b);
        c3 = fma(c3, m, b);
        c4 = fma(c4, m, b);
        c5 = fma(c5, m, b);
        c6 = fma(c6, m, b);
        c7 = fma(c7, m, b);
    }
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = c0 + c1 + c2 + c3 + c4 + c5 + c6 + c7;
}

int grid_cap(int per_cu)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus * per_cu;
}

}  // namespace

extern "C" {

// Copy n16 16-byte elements (device pointers, 16-byte aligned).  0 or the
// hipError_t of the launch.
int pino_probe_copy(const void* src, void* dst, int64_t n16, void* stream)
{
    if (!src || !dst || n16 < 0)
        return (int)hipErrorInvalidValue;
    const int64_t need = (n16 + 1023) / 1024;
    const int grid = (int)(need < grid_cap(16) ? need : grid_cap(16));
    hipLaunchKernelGGL(k_probe_copy, dim3(grid > 0 ? grid : 1), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const i4v*>(src), static_cast<i4v*>(dst), n16);
    return (int)hipGetLastError();
}

// The data movement of the per-radius FP64 kernel over n particles (n even;
// h[6] FP64 SoA, Fmax f64, Rmax i32, all 16-byte aligned).
int pino_probe_stream(const double* const* h, double* Fmax, int32_t* Rmax, int64_t n, int32_t radius,
                      void* stream)
{
    if (!h || !Fmax || !Rmax || n < 0 || (n & 1))
        return (int)hipErrorInvalidValue;
    for (int c = 0; c < 6; ++c)
        if (!h[c])
            return (int)hipErrorInvalidValue;
    const int64_t np = n / 2;
    const int64_t need = (np + 255) / 256;
    const int grid = (int)(need < grid_cap(8) ? need : grid_cap(8));
    hipLaunchKernelGGL(k_probe_stream, dim3(grid > 0 ? grid : 1), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const d2v*>(h[0]), reinterpret_cast<const d2v*>(h[1]),
                       reinterpret_cast<const d2v*>(h[2]), reinterpret_cast<const d2v*>(h[3]),
                       reinterpret_cast<const d2v*>(h[4]), reinterpret_cast<const d2v*>(h[5]),
                       reinterpret_cast<d2v*>(Fmax), reinterpret_cast<int2*>(Rmax), np, radius);
    return (int)hipGetLastError();
}

// blocks x 256 lanes x 8 chains x iters FMAs (2 flops each); out holds
// blocks * 256 doubles.
int pino_probe_fma_f64(double* out, int32_t blocks, int32_t iters, void* stream)
{
    if (!out || blocks <= 0 || iters <= 0)
        return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_probe_fma_f64, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), out, iters,
                       1e-9);
    return (int)hipGetLastError();
}

}  // extern "C"
