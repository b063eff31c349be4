// Host side of include/pino_batch.h.  Included once, by pino_collapse.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/pino_batch.h"
#include "ctx.h"
#include "kernels_batch.h"

struct pino_batch {
    pino_ctx* ctx = nullptr;
    uint32_t flags = 0;
    int32_t n_reals = 0;
    int64_t tile = 0;
    int32_t blocks_per_cu = 0;
    int32_t grid = 0;
    int64_t n_tiles = 0;
    std::vector<pino::RealDesc> host;
    std::vector<int64_t> counts;
    pino::RealDesc* d_reals = nullptr;
    const void** d_ptrs = nullptr;
    pino::Tile* d_tiles = nullptr;
    size_t lds = 0;
    bool f32 = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

pino_status batch_fail(pino_batch* b, hipError_t e, const char* what)
{
    b->ctx->broken = true;
    b->ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return PINO_ERR_HIP;
}

#define BATCH_HIP(b, call)                        \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess)                     \
            return batch_fail((b), e_, #call);    \
    } while (0)

// tiles of `tile` particles (the last one of each realisation shorter)
pino_status batch_tiles(pino_batch* b, int64_t tile)
{
    std::vector<pino::Tile> tiles;
    for (int32_t r = 0; r < b->n_reals; ++r)
        for (int64_t s = 0; s < b->counts[r]; s += tile)
            tiles.push_back(pino::Tile{r, 0, s, std::min(tile, b->counts[r] - s)});
    if (b->d_tiles)
        BATCH_HIP(b, hipFree(b->d_tiles));
    b->d_tiles = nullptr;
    b->n_tiles = (int64_t)tiles.size();
    b->tile = tile;
    if (!tiles.empty()) {
        BATCH_HIP(b, hipMalloc((void**)&b->d_tiles, tiles.size() * sizeof(pino::Tile)));
        BATCH_HIP(b, hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(pino::Tile), hipMemcpyHostToDevice));
    }
    return PINO_OK;
}

pino_status batch_launch(pino_batch* b, hipStream_t st)
{
    if (b->n_tiles == 0)
        return PINO_OK;
    const uint32_t reset = (b->flags & PINO_EVAL_RESET) ? 1u : 0u;
    if (b->f32)
        hipLaunchKernelGGL(pino::k_batch<true>, dim3(b->grid), dim3(256), b->lds, st, b->d_reals, b->d_tiles,
                           b->n_tiles, reset);
    else
        hipLaunchKernelGGL(pino::k_batch<false>, dim3(b->grid), dim3(256), b->lds, st, b->d_reals, b->d_tiles,
                           b->n_tiles, reset);
    BATCH_HIP(b, hipGetLastError());
    return PINO_OK;
}

void batch_release(pino_batch* b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    void* ptrs[] = {b->d_reals, (void*)b->d_ptrs, b->d_tiles};
    for (void* p : ptrs)
        if (p)
            (void)hipFree(p);
}

}  // namespace

extern "C" {

pino_status pino_collapse_batch_plan(pino_ctx* ctx, const pino_realisation* reals, int32_t n_reals, uint32_t flags,
                                     const pino_batch_tuning* tuning, pino_batch** out)
{
    if (!out || !ctx) {
        g_init_error = "ctx and out must be non-NULL";
        return PINO_ERR_ARG;
    }
    *out = nullptr;
    if (ctx->broken)
        return PINO_ERR_STATE;
    auto arg = [&](const std::string& why) {
        ctx->err = why;
        return PINO_ERR_ARG;
    };
    if (ctx->method != PINO_CLASSIC || (ctx->precision != PINO_FP64 && ctx->precision != PINO_MIXED))
        return arg("batched evaluation needs a Classic context in PINO_FP64 or PINO_MIXED");
    if (n_reals < 0 || (n_reals > 0 && !reals))
        return arg("bad realisation array");
    if (flags & ~(PINO_EVAL_RESET | PINO_EVAL_FINALIZE))
        return arg("flags: only PINO_EVAL_RESET and PINO_EVAL_FINALIZE apply");
    if (tuning && (tuning->tile < 0 || tuning->tile % 256 != 0 || tuning->blocks_per_cu < 0 ||
                   tuning->blocks_per_cu > 64))
        return arg("tuning: tile a multiple of 256, 0 <= blocks_per_cu <= 64");
    for (int32_t r = 0; r < n_reals; ++r) {
        const pino_realisation& R = reals[r];
        const std::string at = "realisation " + std::to_string(r) + ": ";
        if (R.n < 0 || R.n_radii < 1 || R.cosmo < 0 || R.cosmo >= ctx->n_cosmo || R.radius_offset < 0)
            return arg(at + "need n >= 0, n_radii >= 1, a valid cosmo and radius_offset >= 0");
        if (R.n == 0)
            continue;
        if (!R.h || !R.Fmax || !R.Rmax)
            return arg(at + "h, Fmax and Rmax must be non-NULL");
        for (int k = 0; k < 6 * R.n_radii; ++k)
            if (!R.h[k])
                return arg(at + "NULL Hessian component pointer");
        if ((flags & PINO_EVAL_FINALIZE) && !R.a_coll)
            return arg(at + "PINO_EVAL_FINALIZE needs a_coll");
    }
    pino_batch* b = new (std::nothrow) pino_batch();
    if (!b)
        return PINO_ERR_ALLOC;
    b->ctx = ctx;
    b->flags = flags;
    b->n_reals = n_reals;
    b->f32 = ctx->precision == PINO_MIXED;
    auto fail = [&](pino_status s) {
        batch_release(b);
        delete b;
        return s;
    };
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->err = "hipSetDevice failed";
        return fail(PINO_ERR_HIP);
    }
    // pointer arrays of every realisation, concatenated
    std::vector<const void*> ptrs;
    std::vector<size_t> first;
    for (int32_t r = 0; r < n_reals; ++r) {
        first.push_back(ptrs.size());
        for (int k = 0; k < 6 * reals[r].n_radii; ++k)
            ptrs.push_back(reals[r].n > 0 ? reals[r].h[k] : nullptr);
    }
    hipError_t e = hipSuccess;
    if (!ptrs.empty()) {
        e = hipMalloc((void**)&b->d_ptrs, ptrs.size() * sizeof(void*));
        if (e == hipSuccess)
            e = hipMemcpy(b->d_ptrs, ptrs.data(), ptrs.size() * sizeof(void*), hipMemcpyHostToDevice);
    }
    int nk_max = 0, nb_max = 0;
    for (int32_t r = 0; r < n_reals; ++r) {
        const pino_realisation& R = reals[r];
        pino::RealDesc d{};
        d.n = R.n;
        d.n_radii = R.n_radii;
        d.cosmo = R.cosmo;
        d.radius_offset = R.radius_offset;
        d.nk = ctx->nk[R.cosmo];
        d.h = b->d_ptrs + first[r];
        d.Fmax = R.Fmax;
        d.Rmax = R.Rmax;
        d.acoll = (flags & PINO_EVAL_FINALIZE) ? R.a_coll : nullptr;
        d.growth = ctx->d_growth + (size_t)R.cosmo * 3 * ctx->nk_max;
        d.growth32 = ctx->d_growth32 ? ctx->d_growth32 + (size_t)R.cosmo * 3 * ctx->nk_max : nullptr;
        // two particles per lane need every Hessian array aligned to two
        // elements, Fmax and a_coll to 16 bytes and Rmax to 8
        {
            const uintptr_t two = ctx->precision == PINO_FP64 ? 16 : 8;
            auto al = [](const void* p, uintptr_t b) { return reinterpret_cast<uintptr_t>(p) % b == 0; };
            bool ok = al(R.Fmax, 16) && al(R.Rmax, 8) && (!d.acoll || al(d.acoll, 16));
            for (int k = 0; R.n > 0 && k < 6 * R.n_radii; ++k)
                ok = ok && al(R.h[k], two);
            d.paired = ok ? 1 : 0;
        }
        d.gi.idx = ctx->d_gidx + (size_t)R.cosmo * 2 * ctx->nb_max;
        d.gi.nb = ctx->nb[R.cosmo];
        d.gi.L0 = ctx->gL0[R.cosmo];
        d.gi.S = ctx->gS[R.cosmo];
        d.gi.ok = ctx->gok[R.cosmo];
        b->host.push_back(d);
        b->counts.push_back(R.n);
        nk_max = std::max(nk_max, d.nk);
        nb_max = std::max(nb_max, d.gi.nb);
    }
    if (e == hipSuccess && n_reals > 0) {
        e = hipMalloc((void**)&b->d_reals, b->host.size() * sizeof(pino::RealDesc));
        if (e == hipSuccess)
            e = hipMemcpy(b->d_reals, b->host.data(), b->host.size() * sizeof(pino::RealDesc), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        ctx->broken = true;
        ctx->err = std::string("batch plan: ") + hipGetErrorString(e);
        return fail(PINO_ERR_HIP);
    }
    b->lds = b->f32 ? pino::growth32_lds_bytes(nk_max, nb_max) : pino::growth_lds_bytes(nk_max, nb_max);

    int64_t tile = tuning && tuning->tile > 0 ? tuning->tile : 8192;
    int32_t bpc = tuning && tuning->blocks_per_cu > 0 ? tuning->blocks_per_cu : 8;
    if (tuning && tuning->autotune && n_reals > 0) {
        // time each candidate on the real data (each run overwrites the outputs
        // with the same values) and keep the fastest
        const int64_t tiles[] = {2048, 8192, 32768};
        const int32_t bpcs[] = {4, 8, 16};
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            ctx->err = "hipEventCreate failed";
            return fail(PINO_ERR_HIP);
        }
        float best = 1e30f;
        int64_t best_tile = tile;
        int32_t best_bpc = bpc;
        for (int64_t tcand : tiles)
            for (int32_t bcand : bpcs) {
                if (batch_tiles(b, tcand) != PINO_OK)
                    return fail(PINO_ERR_HIP);
                b->grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)ctx->cu_count * bcand, b->n_tiles));
                b->blocks_per_cu = bcand;
                float ms = 0.0f;
                pino_status s = batch_launch(b, nullptr);  // warm-up
                if (s == PINO_OK && hipEventRecord(e0, nullptr) == hipSuccess && (s = batch_launch(b, nullptr)) == PINO_OK &&
                    hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                    hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
                    if (ms < best) {
                        best = ms;
                        best_tile = tcand;
                        best_bpc = bcand;
                    }
                } else {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return fail(s != PINO_OK ? s : PINO_ERR_HIP);
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        tile = best_tile;
        bpc = best_bpc;
    }
    if (batch_tiles(b, tile) != PINO_OK)
        return fail(PINO_ERR_HIP);
    b->blocks_per_cu = bpc;
    b->grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)ctx->cu_count * bpc, std::max<int64_t>(b->n_tiles, 1)));
    *out = b;
    return PINO_OK;
}

pino_status pino_collapse_batch_run(pino_batch* b, void* hip_stream)
{
    if (!b)
        return PINO_ERR_ARG;
    if (b->ctx->broken)
        return PINO_ERR_STATE;
    BATCH_HIP(b, hipSetDevice(b->ctx->device));
    return batch_launch(b, static_cast<hipStream_t>(hip_stream));
}

pino_status pino_collapse_batch_graph_launch(pino_batch* b, void* hip_stream)
{
    if (!b || !hip_stream) {
        if (b)
            b->ctx->err = "graph launch needs a non-NULL stream";
        return PINO_ERR_ARG;
    }
    if (b->ctx->broken)
        return PINO_ERR_STATE;
    BATCH_HIP(b, hipSetDevice(b->ctx->device));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (!b->exec) {
        BATCH_HIP(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const pino_status s = batch_launch(b, st);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (s != PINO_OK)
            return s;
        if (e != hipSuccess)
            return batch_fail(b, e, "hipStreamEndCapture");
        b->graph = g;
        BATCH_HIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    BATCH_HIP(b, hipGraphLaunch(b->exec, st));
    return PINO_OK;
}

pino_status pino_collapse_batch_config(const pino_batch* b, int64_t* tile, int32_t* blocks_per_cu, int32_t* grid,
                                       int64_t* n_tiles)
{
    if (!b)
        return PINO_ERR_ARG;
    if (tile)
        *tile = b->tile;
    if (blocks_per_cu)
        *blocks_per_cu = b->blocks_per_cu;
    if (grid)
        *grid = b->grid;
    if (n_tiles)
        *n_tiles = b->n_tiles;
    return PINO_OK;
}

pino_status pino_collapse_batch_free(pino_batch* b)
{
    if (!b)
        return PINO_OK;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    batch_release(b);
    delete b;
    return PINO_OK;
}

}  // extern "C"
