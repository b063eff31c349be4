// Hessian stage: the six weighted copies of delta(k) whose inverse real FFTs
// are the second derivatives of the smoothed potential (Sec. 3: Poisson
// equation, Gaussian smoothing, derivatives by FFT).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pino {

// Signed FFT frequency index of position i on a side of n (0, 1, ...,
// -n/2 at the Nyquist position of an even side, ..., -1).
__device__ __forceinline__ int fft_freq(int i, int n)
{
    return i < (n + 1) / 2 ? i : i - n;
}

// One thread per mode m = (ix * n + iy) * nz + iz of the half grid
// (nz = n/2 + 1): reads delta(k) once and writes, for the component pairs
// (xx, yy, zz, xy, xz, yz), delta(k) k_i k_j exp(-k^2 R^2/2) / (k^2 n^3)
// to out[c * modes + m] (0 at k = 0 and at Nyquist indices).  The 1/n^3 is
// the normalisation of the inverse transform, which the FFT library leaves
// out.  C2 is double2 (FP64 stage) or float2 (FP32 stage); the weights are
// formed in FP64.
template <typename C2>
__global__ void __launch_bounds__(256) k_hessian_modes(const double2* __restrict__ dk, int n, int nz, double kf,
                                                      double R, double inv_n3, C2* __restrict__ out)
{
    const int64_t modes = (int64_t)n * n * nz;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= modes)
        return;
    const int iz = (int)(m % nz);
    const int64_t row = m / nz;
    const int iy = (int)(row % n);
    const int ix = (int)(row / n);
    const double kx = kf * fft_freq(ix, n);
    const double ky = kf * fft_freq(iy, n);
    const double kz = kf * iz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    // k = 0 and, for an even side, the Nyquist index along any axis (where
    // +n/2 and -n/2 alias and a derivative is not defined) are dropped
    const bool nyq = (n % 2 == 0) && (2 * ix == n || 2 * iy == n || 2 * iz == n);
    const double w = (k2 > 0.0 && !nyq) ? exp(-0.5 * k2 * R * R) / k2 * inv_n3 : 0.0;
    const double2 d = dk[m];
    const double re = d.x * w, im = d.y * w;
    const double kk[6] = {kx * kx, ky * ky, kz * kz, kx * ky, kx * kz, ky * kz};
    for (int c = 0; c < 6; ++c) {
        C2 v;
        v.x = re * kk[c];
        v.y = im * kk[c];
        out[c * modes + m] = v;
    }
}

}  // namespace pino
