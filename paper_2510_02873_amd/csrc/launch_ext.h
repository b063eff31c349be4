// Launchers of the reduced-precision and surrogate variants.
#pragma once

#include "ctx.h"
#include "kernels_fp64.h"

namespace {

inline bool mlp_blob_valid(const void*, int64_t, std::string& why)
{
    why = "not available";
    return false;
}

inline pino_status mlp_upload(pino_ctx* c, const void*, int64_t)
{
    c->err = "surrogate not available";
    return PINO_ERR_UNSUPPORTED;
}

inline pino_status launch_mixed(pino_ctx* c, const pino_item&, const pino::ItemArgs&, uint32_t, hipStream_t, int,
                                int)
{
    c->err = "mixed precision not available";
    return PINO_ERR_UNSUPPORTED;
}

inline pino_status launch_surrogate(pino_ctx* c, const pino_item&, const pino::ItemArgs&, uint32_t, hipStream_t,
                                    int, int)
{
    c->err = "surrogate not available";
    return PINO_ERR_UNSUPPORTED;
}

}  // namespace
