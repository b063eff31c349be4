// Launcher of the mixed-precision variant.
#pragma once

#include "ctx.h"
#include "kernels_fp64.h"
#include "kernels_mixed.h"

namespace {



inline pino_status launch_mixed(pino_ctx* c, const pino_item& it, const pino::ItemArgs& a, uint32_t, hipStream_t st,
                                int grid, int block)
{
    if (c->method != PINO_CLASSIC) {
        c->err = "mixed precision is implemented for the Classic method";
        return PINO_ERR_UNSUPPORTED;
    }
    const float* g32 = c->d_growth32 + (size_t)it.cosmo * 3 * c->nk_max;
    const size_t lds = pino::growth32_lds_bytes(a.nk, a.gi.nb);
    hipLaunchKernelGGL(pino::k_classic_mixed, dim3(grid), dim3(block), lds, st, a, g32);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->broken = true;
        c->err = std::string("k_classic_mixed launch: ") + hipGetErrorString(e);
        return PINO_ERR_HIP;
    }
    return PINO_OK;
}


}  // namespace
