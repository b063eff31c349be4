// Stand-alone evaluation kernels of the interpolators (Sec. 4.3 benchmarks):
// the same device functions the collapse kernels use, on given queries.
#pragma once

#include "kernels_fp64.h"

namespace pino {

// Natural-spline values at m queries; the n knots (x, y, M) are staged in
// LDS once per workgroup (grid-stride loop over queries).
__global__ void __launch_bounds__(256) k_spline_eval(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ M, int n,
                                                    const double* __restrict__ q, double* __restrict__ out,
                                                    int64_t m)
{
    extern __shared__ double lds[];
    double* xs = lds;
    double* ys = xs + n;
    double* ms = ys + n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        xs[k] = x[k];
        ys[k] = y[k];
        ms[k] = M[k];
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const double v = q[i];
        const int j = locate(xs, n, v);
        out[i] = spline_piece(xs[j], xs[j + 1], ys[j], ys[j + 1], ms[j], ms[j + 1], v);
    }
}

// The Tabulated interpolator at m queries (x, y, d); knots in LDS, the
// interleaved (F, M) table read from global memory (L2-resident).
__global__ void __launch_bounds__(256) k_table_eval(TabArgs t, const double* __restrict__ qx,
                                                   const double* __restrict__ qy, const double* __restrict__ qd,
                                                   double* __restrict__ out, int64_t m)
{
    extern __shared__ double lds[];
    double* xs = lds;
    double* ys = xs + t.nx;
    double* ds = ys + t.ny;
    const int* idx = stage_table(xs, t);
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
        out[i] = table_at(t, xs, ys, ds, idx, qx[i], qy[i], qd[i]);
}

}  // namespace pino
