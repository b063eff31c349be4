// Stand-alone evaluation kernels of the interpolators (Sec. 4.3 benchmarks):
// the same device functions the collapse kernels use, on given queries.
#pragma once

#include "kernels_fp64.h"

namespace pino {

// Natural-spline values at m queries; the n knots (x, y, M) are staged in
// LDS once per workgroup (grid-stride loop over queries).  With nb > 0 the
// block also builds an interval index of nb bins in LDS (build_axis_index)
// and, where it holds, finds each query's interval from its bin; otherwise
// (nb = 0, or the knots cluster too much) by binary search.  The interval is
// the same either way.
__global__ void __launch_bounds__(256) k_spline_eval(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ M, int n, int nb,
                                                    const double* __restrict__ q, double* __restrict__ out,
                                                    int64_t m)
{
    extern __shared__ double lds[];
    double* xs = lds;
    double* ys = xs + n;
    double* ms = ys + n;
    int* idx = reinterpret_cast<int*>(ms + n);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        xs[k] = x[k];
        ys[k] = y[k];
        ms[k] = M[k];
    }
    __syncthreads();
    double bpu = 0.0;
    const bool indexed = nb > 0 && build_axis_index<kIndexCompares + 1>(xs, n, nb, idx, bpu);
    const double lo = xs[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const double v = q[i];
        int j;
        if (indexed) {
            const double fb = fmin(fmax((v - lo) * bpu, 0.0), (double)(nb - 1));
            j = locate_after<kIndexCompares + 1>(xs, n, v, idx[(int)fb]);
        } else {
            j = locate(xs, n, v);
        }
        out[i] = spline_piece(xs[j], xs[j + 1], ys[j], ys[j + 1], ms[j], ms[j + 1], v);
    }
}

// The Tabulated interpolator at m queries (x, y, d); knots in LDS, the
// interleaved (F, M) table read from global memory (L2-resident).  The
// intervals are found by binary search: a per-block index (as the spline
// has) measured slower here, the four corner gathers dominating.
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
