// Reduced-precision building blocks: FP32 eigenvalues and FP32 natural-spline
// interpolation, used by the mixed-precision path together with the FP64
// collapse root of device_collapse.h.
#pragma once

#include "device_collapse.h"

namespace pino {

struct Hess32 {
    float xx, yy, zz, xy, xz, yz;
};

__host__ __device__ __forceinline__ Hess64 widen(const Hess32& h)
{
    return Hess64{h.xx, h.yy, h.zz, h.xy, h.xz, h.yz};
}

// Threshold on 1 + r below which the FP32 closed form is not trusted for l1
// (l1 ~ l2: its FP32 error grows like eps * p^2 / (l1 - l2)); such lanes take
// the FP64 eigenvalue path on the same (widened) inputs.
constexpr float kNearRepeated32 = 1e-3f;

// FP32 largest eigenvalue with s = l2 + l3 and pp = l2 l3 (see eig_top);
// returns false when the FP64 path must decide.
__host__ __device__ __forceinline__ bool eig_top_f32(const Hess32& h, float& l1, float& s, float& pp)
{
    const float tr = h.xx + h.yy + h.zz;
    const float q = tr * (1.0f / 3.0f);
    const float dx = h.xx - q, dy = h.yy - q, dz = h.zz - q;
    const float off = h.xy * h.xy + h.xz * h.xz + h.yz * h.yz;
    const float ss = dx * dx + dy * dy + dz * dz + 2.0f * off;
    const float p = sqrtf(ss * (1.0f / 6.0f));
    const float det = dx * (dy * dz - h.yz * h.yz) - h.xy * (h.xy * dz - h.yz * h.xz) + h.xz * (h.xy * h.yz - dy * h.xz);
    const float ip = p > 0.0f ? 1.0f / p : 0.0f;
    float r = 0.5f * det * (ip * ip * ip);
    r = fminf(fmaxf(r, -1.0f), 1.0f);
    l1 = q + 2.0f * p * cos_acos3(0.5f + 0.5f * r);
    const float mu2 = h.xx * h.yy + h.xx * h.zz + h.yy * h.zz - off;
    s = tr - l1;
    pp = mu2 - l1 * s;
    return 1.0f + r >= kNearRepeated32;
}

// All three eigenvalues in FP32, descending: l1 and l3 from the closed form
// (the smallest root of x^3 - 3x = 2r is minus the largest root for -r), l2
// from the trace.  Returns false when a pair is nearly repeated at either end
// of r (1 -/+ r below kNearRepeated32), where the FP32 closed form loses the
// pair's digits; the FP64 path (eig_all, with its deflation) decides those.
__host__ __device__ __forceinline__ bool eig_all_f32(const Hess32& h, float& l1, float& l2, float& l3)
{
    const float tr = h.xx + h.yy + h.zz;
    const float q = tr * (1.0f / 3.0f);
    const float dx = h.xx - q, dy = h.yy - q, dz = h.zz - q;
    const float off = h.xy * h.xy + h.xz * h.xz + h.yz * h.yz;
    const float ss = dx * dx + dy * dy + dz * dz + 2.0f * off;
    const float p = sqrtf(ss * (1.0f / 6.0f));
    const float det = dx * (dy * dz - h.yz * h.yz) - h.xy * (h.xy * dz - h.yz * h.xz) + h.xz * (h.xy * h.yz - dy * h.xz);
    const float ip = p > 0.0f ? 1.0f / p : 0.0f;
    float r = 0.5f * det * (ip * ip * ip);
    r = fminf(fmaxf(r, -1.0f), 1.0f);
    l1 = q + 2.0f * p * cos_acos3(0.5f + 0.5f * r);
    l3 = q - 2.0f * p * cos_acos3(0.5f - 0.5f * r);
    l2 = fminf(fmaxf(tr - l1 - l3, l3), l1);
    return 1.0f + r >= kNearRepeated32 && 1.0f - r >= kNearRepeated32;
}

// Natural-spline piece in FP32 (as spline_piece).
__host__ __device__ __forceinline__ float spline_piece32(float x0, float x1, float y0, float y1, float m0, float m1,
                                                  float q)
{
    const float h = x1 - x0;
    const float t = (q - x0) / h;
    const float w = 1.0f - t;
    return w * y0 + t * y1 + (h * h * (1.0f / 6.0f)) * ((w * w * w - w) * m0 + (t * t * t - t) * m1);
}

// a(D) through the natural spline with FP32 knots [D | a | M] (n each) and the
// same interval index as the FP64 path.
__host__ __device__ __forceinline__ int locate32(const float* x, int n, float q)
{
    int lo = 0;
    int step = 1;
    while (step * 2 <= n - 2)
        step *= 2;
    for (; step > 0; step >>= 1) {
        const int j = lo + step;
        if (j <= n - 2 && x[j] <= q)
            lo = j;
    }
    return lo;
}

__host__ __device__ __forceinline__ float growth_invert_f32(const float* g, int n, float Dc, const GrowthIndex& gi)
{
    const float* D = g;
    const float* a = g + n;
    const float* M = g + 2 * n;
    if (!(Dc <= D[n - 1]))
        return __builtin_huge_valf();
    if (Dc < D[0])
        return a[0];
    int i;
    if (gi.ok) {
        float fb = (__log2f(Dc) - gi.L0) * gi.S;
        fb = fminf(fmaxf(fb, 0.0f), (float)(gi.nb - 1));
        i = gi.idx[(int)fb];
        i += (i + 1 <= n - 2 && D[i + 1] <= Dc) ? 1 : 0;
        i += (i + 1 <= n - 2 && D[i + 1] <= Dc) ? 1 : 0;
    } else {
        i = locate32(D, n, Dc);
    }
    const float h = D[i + 1] - D[i];
    const float t = (Dc - D[i]) / h;
    const float w = 1.0f - t;
    return w * a[i] + t * a[i + 1] + (h * h * (1.0f / 6.0f)) * ((w * w * w - w) * M[i] + (t * t * t - t) * M[i + 1]);
}

}  // namespace pino
