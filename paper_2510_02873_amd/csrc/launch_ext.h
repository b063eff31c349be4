// Launcher of the mixed-precision variant.
#pragma once

#include "ctx.h"
#include "kernels_fp64.h"
#include "kernels_mixed.h"

namespace {



// tab: the Tabulated kernels' view of this radius' table (NULL for Classic)
inline pino_status launch_mixed(pino_ctx* c, const pino_item& it, const pino::ItemArgs& a, const pino::TabArgs* tab,
                                hipStream_t st, int grid, int block)
{
    const float* g32 = c->d_growth32 + (size_t)it.cosmo * 3 * c->nk_max;
    const size_t lds = pino::growth32_lds_bytes(a.nk, a.gi.nb);
    // pairs of particles per lane need 8-byte aligned FP32 components,
    // 16-byte aligned Fmax and a_coll and an 8-byte aligned Rmax
    auto al = [](const void* p, uintptr_t b) { return reinterpret_cast<uintptr_t>(p) % b == 0; };
    bool paired = al(a.Fmax, 16) && al(a.Rmax, 8) && (!a.acoll || al(a.acoll, 16));
    for (int k = 0; k < 6; ++k)
        paired = paired && al(a.h[k], 8);
    const int64_t need = (a.n / 2 + block - 1) / block;
    const int gp = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)c->cu_count * c->blocks_per_cu));
    if (tab) {
        const auto* t32 = static_cast<const pino::f4v*>(c->d_tab32);
        const size_t lds_t = lds + pino::table_lds_bytes(*tab);
        if (paired)
            hipLaunchKernelGGL(pino::k_tabulated_mixed, dim3(gp), dim3(block), lds_t, st, a, *tab, t32, g32);
        else
            hipLaunchKernelGGL(pino::k_tabulated_mixed_1, dim3(grid), dim3(block), lds_t, st, a, *tab, t32, g32);
    } else if (paired) {
        hipLaunchKernelGGL(pino::k_classic_mixed, dim3(gp), dim3(block), lds, st, a, g32);
    } else {
        hipLaunchKernelGGL(pino::k_classic_mixed_1, dim3(grid), dim3(block), lds, st, a, g32);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->broken = true;
        c->err = std::string(tab ? "k_tabulated_mixed" : "k_classic_mixed") + " launch: " + hipGetErrorString(e);
        return PINO_ERR_HIP;
    }
    return PINO_OK;
}


}  // namespace
