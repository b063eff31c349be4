// pino_field.h implementation: Hessians from delta(k) with hipFFT, and the
// collapse of a radius list fed from them on the device.
#pragma once

#include <hipfft/hipfft.h>

#include <string>

#include "../../include/pino_field.h"
#include "ctx.h"
#include "kernels_field.h"

struct pino_field {
    int device = 0;
    int n = 0;
    int nz = 0;
    double box = 0.0;
    int64_t modes = 0;    // n * n * nz
    int64_t points = 0;   // n^3
    void* kbuf = nullptr;       // 6 * modes complex128 (or complex64 for FP32)
    double* hbuf = nullptr;     // 6 * points doubles (or floats for FP32)
    hipfftHandle p64 = 0, p32 = 0;
    bool has64 = false, has32 = false;
    StreamOrder order;  // kbuf and hbuf are shared by every call on the field
    bool broken = false;
    std::string err = "no error";
};

namespace {

thread_local std::string g_field_error = "no error";

const char* hipfft_name(hipfftResult r)
{
    switch (r) {
    case HIPFFT_SUCCESS: return "HIPFFT_SUCCESS";
    case HIPFFT_INVALID_PLAN: return "HIPFFT_INVALID_PLAN";
    case HIPFFT_ALLOC_FAILED: return "HIPFFT_ALLOC_FAILED";
    case HIPFFT_INVALID_VALUE: return "HIPFFT_INVALID_VALUE";
    case HIPFFT_INTERNAL_ERROR: return "HIPFFT_INTERNAL_ERROR";
    case HIPFFT_EXEC_FAILED: return "HIPFFT_EXEC_FAILED";
    case HIPFFT_SETUP_FAILED: return "HIPFFT_SETUP_FAILED";
    case HIPFFT_INVALID_SIZE: return "HIPFFT_INVALID_SIZE";
    default: return "hipFFT error";
    }
}

pino_status field_fail(pino_field* f, const std::string& what)
{
    f->broken = true;
    f->err = what;
    return PINO_ERR_HIP;
}

#define FIELD_HIP(f, call)                                                        \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return field_fail((f), std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define FIELD_FFT(f, call)                                             \
    do {                                                               \
        hipfftResult r_ = (call);                                      \
        if (r_ != HIPFFT_SUCCESS)                                      \
            return field_fail((f), std::string(#call) + ": " + hipfft_name(r_)); \
    } while (0)

void field_release(pino_field* f)
{
    if (f->has64)
        (void)hipfftDestroy(f->p64);
    if (f->has32)
        (void)hipfftDestroy(f->p32);
    if (f->kbuf)
        (void)hipFree(f->kbuf);
    if (f->hbuf)
        (void)hipFree(f->hbuf);
    f->has64 = f->has32 = false;
    f->kbuf = nullptr;
    f->hbuf = nullptr;
    f->order.destroy();
}

pino_status field_init(pino_field* f)
{
    FIELD_HIP(f, hipSetDevice(f->device));
    FIELD_HIP(f, hipMalloc(&f->kbuf, (size_t)6 * f->modes * sizeof(double2)));
    FIELD_HIP(f, hipMalloc((void**)&f->hbuf, (size_t)6 * f->points * sizeof(double)));
    int dims[3] = {f->n, f->n, f->n};
    int inembed[3] = {f->n, f->n, f->nz};
    int onembed[3] = {f->n, f->n, f->n};
    // six transforms per call, one per component, back to back in memory
    FIELD_FFT(f, hipfftPlanMany(&f->p64, 3, dims, inembed, 1, (int)f->modes, onembed, 1, (int)f->points,
                                HIPFFT_Z2D, 6));
    f->has64 = true;
    FIELD_FFT(f, hipfftPlanMany(&f->p32, 3, dims, inembed, 1, (int)f->modes, onembed, 1, (int)f->points,
                                HIPFFT_C2R, 6));
    f->has32 = true;
    FIELD_HIP(f, f->order.create());
    return PINO_OK;
}

// delta(k) -> six weighted copies in kbuf -> six inverse real transforms
template <bool F32>
pino_status field_hessian_impl(pino_field* f, const void* delta_k, double R, void* H, hipStream_t st)
{
    FIELD_HIP(f, hipSetDevice(f->device));
    const double kf = 2.0 * M_PI / f->box;
    const double inv_n3 = 1.0 / (double)f->points;
    const unsigned blocks = (unsigned)((f->modes + 255) / 256);
    const auto* dk = static_cast<const double2*>(delta_k);
    if (F32) {
        hipLaunchKernelGGL(pino::k_hessian_modes<float2>, dim3(blocks), dim3(256), 0, st, dk, f->n, f->nz, kf, R,
                           inv_n3, static_cast<float2*>(f->kbuf));
        FIELD_HIP(f, hipGetLastError());
        FIELD_FFT(f, hipfftSetStream(f->p32, st));
        FIELD_FFT(f, hipfftExecC2R(f->p32, static_cast<hipfftComplex*>(f->kbuf), static_cast<hipfftReal*>(H)));
    } else {
        hipLaunchKernelGGL(pino::k_hessian_modes<double2>, dim3(blocks), dim3(256), 0, st, dk, f->n, f->nz, kf, R,
                           inv_n3, static_cast<double2*>(f->kbuf));
        FIELD_HIP(f, hipGetLastError());
        FIELD_FFT(f, hipfftSetStream(f->p64, st));
        FIELD_FFT(f, hipfftExecZ2D(f->p64, static_cast<hipfftDoubleComplex*>(f->kbuf),
                                   static_cast<hipfftDoubleReal*>(H)));
    }
    return PINO_OK;
}

pino_status field_check(pino_field* f, const void* delta_k, double R, const void* H)
{
    if (f->broken)
        return PINO_ERR_STATE;
    if (!delta_k || !H || !(R >= 0.0) || !std::isfinite(R)) {
        f->err = "delta_k and H must be non-NULL and R finite and >= 0";
        return PINO_ERR_ARG;
    }
    return PINO_OK;
}

}  // namespace

extern "C" {

pino_status pino_field_create(int32_t device, int32_t n_side, double box, pino_field** out)
{
    if (!out) {
        g_field_error = "out is NULL";
        return PINO_ERR_ARG;
    }
    *out = nullptr;
    if (device < 0 || n_side < 2 || n_side > 1024 || !(box > 0.0) || !std::isfinite(box)) {
        g_field_error = "need device >= 0, 2 <= n_side <= 1024 and a finite box > 0";
        return PINO_ERR_ARG;
    }
    pino_field* f = new (std::nothrow) pino_field();
    if (!f) {
        g_field_error = "out of host memory";
        return PINO_ERR_ALLOC;
    }
    f->device = device;
    f->n = n_side;
    f->nz = n_side / 2 + 1;
    f->box = box;
    f->modes = (int64_t)n_side * n_side * f->nz;
    f->points = (int64_t)n_side * n_side * n_side;
    const pino_status st = field_init(f);
    if (st != PINO_OK) {
        g_field_error = f->err;
        field_release(f);
        delete f;
        return st;
    }
    *out = f;
    return PINO_OK;
}

pino_status pino_field_hessian(pino_field* f, const void* delta_k, double R, double* H, void* hip_stream)
{
    if (!f) {
        g_field_error = "field is NULL";
        return PINO_ERR_ARG;
    }
    const pino_status st = field_check(f, delta_k, R, H);
    if (st != PINO_OK)
        return st;
    const hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    FIELD_HIP(f, f->order.enter(hs));
    const pino_status ps = field_hessian_impl<false>(f, delta_k, R, H, hs);
    if (ps != PINO_OK)
        return ps;
    FIELD_HIP(f, f->order.leave(hs));
    return PINO_OK;
}

pino_status pino_field_hessian_f32(pino_field* f, const void* delta_k, double R, float* H, void* hip_stream)
{
    if (!f) {
        g_field_error = "field is NULL";
        return PINO_ERR_ARG;
    }
    const pino_status st = field_check(f, delta_k, R, H);
    if (st != PINO_OK)
        return st;
    const hipStream_t hs = static_cast<hipStream_t>(hip_stream);
    FIELD_HIP(f, f->order.enter(hs));
    const pino_status ps = field_hessian_impl<true>(f, delta_k, R, H, hs);
    if (ps != PINO_OK)
        return ps;
    FIELD_HIP(f, f->order.leave(hs));
    return PINO_OK;
}

pino_status pino_field_collapse(pino_field* f, pino_ctx* ctx, const void* delta_k, const double* radii,
                                const pino_item* items, int32_t n_radii, uint32_t flags, void* hip_stream)
{
    if (!f || !ctx) {
        g_field_error = "field and ctx must be non-NULL";
        return PINO_ERR_ARG;
    }
    if (f->broken)
        return PINO_ERR_STATE;
    if (!delta_k || n_radii < 0 || (n_radii > 0 && (!radii || !items)) ||
        (flags & ~(uint32_t)(PINO_EVAL_RESET | PINO_EVAL_SYNC | PINO_EVAL_FINALIZE))) {
        f->err = "bad arguments (delta_k, radii, items, n_radii or flags)";
        return PINO_ERR_ARG;
    }
    if (ctx->device != f->device) {
        f->err = "the context and the field are on different devices";
        return PINO_ERR_ARG;
    }
    // FP32 Hessians for a mixed-precision context, FP64 otherwise
    const bool f32 = ctx->precision == PINO_MIXED;
    for (int32_t r = 0; r < n_radii; ++r) {
        if (!(radii[r] >= 0.0) || !std::isfinite(radii[r])) {
            f->err = "radii must be finite and >= 0";
            return PINO_ERR_ARG;
        }
        if (items[r].n != f->points) {
            f->err = "every item must cover the field's n^3 particles";
            return PINO_ERR_ARG;
        }
    }
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    FIELD_HIP(f, f->order.enter(st));
    for (int32_t r = 0; r < n_radii; ++r) {
        pino_status ps = f32 ? field_hessian_impl<true>(f, delta_k, radii[r], f->hbuf, st)
                             : field_hessian_impl<false>(f, delta_k, radii[r], f->hbuf, st);
        if (ps != PINO_OK)
            return ps;
        pino_item it = items[r];
        const size_t es = f32 ? sizeof(float) : sizeof(double);
        for (int c = 0; c < 6; ++c)
            it.h[c] = reinterpret_cast<const char*>(f->hbuf) + (size_t)c * f->points * es;
        uint32_t fl = 0;
        if (r == 0)
            fl |= flags & PINO_EVAL_RESET;
        if (r == n_radii - 1)
            fl |= flags & (PINO_EVAL_FINALIZE | PINO_EVAL_SYNC);
        ps = pino_collapse_eval(ctx, &it, 1, fl, hip_stream);
        if (ps != PINO_OK) {
            f->err = std::string("radius ") + std::to_string(r) + ": " + pino_collapse_last_error(ctx);
            return ps;
        }
    }
    FIELD_HIP(f, f->order.leave(st));
    return PINO_OK;
}

pino_status pino_field_free(pino_field* f)
{
    if (!f)
        return PINO_OK;
    if (f->device >= 0)
        (void)hipSetDevice(f->device);
    field_release(f);
    delete f;
    return PINO_OK;
}

const char* pino_field_last_error(const pino_field* f)
{
    return f ? f->err.c_str() : g_field_error.c_str();
}

}  // extern "C"
