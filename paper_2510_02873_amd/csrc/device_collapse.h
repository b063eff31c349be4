// Device building blocks of the collapse-time path (gfx950).
//
// eig_*      : eigenvalues of the 3x3 symmetric Hessian by the trigonometric
//              closed form of the characteristic cubic (Sec. 3: an analytic
//              method, eigenvalues sorted in descending order).
// lpt_root_* : smallest positive root of the axis-1 third-order LPT collapse
//              cubic (Sec. 3), solved in u = l1 * D by a bracketed Halley
//              iteration; the bracket comes from the critical points of the
//              cubic so the root returned is the first crossing.
// spline_*   : natural cubic spline evaluation with knots staged in LDS and a
//              branch-free binary search (Sec. 4.2).
//
// Every function is straight-line code or a loop with a per-lane exit, so
// lanes of a wavefront follow the same instruction stream (Sec. 4.1: masked
// execution instead of divergent branches).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pino {

constexpr double kTwoPiOver3 = 2.0943951023931954923;
constexpr double kInf = __builtin_huge_val();

// Reciprocal: hardware estimate refined by Newton-Raphson steps (each step
// squares the relative error).  Two steps reach the FP64 rounding level; the
// result is not IEEE-rounded, which only the last bit can tell.
__host__ __device__ __forceinline__ double rcp2(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// 1/sqrt(x) for normal x > 0: hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - x y^2)/2 (each squares the relative
// error).
__host__ __device__ __forceinline__ double rsq2(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// One refinement step: enough where the reciprocal scales a small
// correction (a Newton or Halley step), whose own error it then barely moves.
__host__ __device__ __forceinline__ double rcp1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// cos(acos(r)/3) for r in [-1, 1], given h = (1 + r)/2 (which callers form in
// FP64, so that it keeps its digits next to r = -1).  As a function of
// t = sqrt(h) = cos(acos(r)/2) it is cos(2 acos(t)/3), analytic on [0, 1]
// (the square-root branch point of c(r) at r = -1 becomes a regular point),
// so a degree-7 polynomial in t holds it to 2.8e-8 relative (coefficients
// from gen_cos_acos3.py); with FP32 rounding the result is within ~1e-7.
__host__ __device__ __forceinline__ float cos_acos3(float h)
{
    const float t = sqrtf(fmaxf(h, 0.0f));
    float c = 0.0012316048973092788f;
    c = fmaf(c, t, -0.0064512453556797196f);
    c = fmaf(c, t, 0.016541704297467527f);
    c = fmaf(c, t, -0.030569944240758228f);
    c = fmaf(c, t, 0.052957431674725962f);
    c = fmaf(c, t, -0.11105763313282863f);
    c = fmaf(c, t, 0.57734809605336668f);
    return fmaf(c, t, 0.50000001420359497f);
}

// x = 2 cos(phi), the root of x^3 - 3x = 2r on [1, 2] (phi = acos(r)/3, the
// largest eigenvalue) or on [-2, -1] (phi + 2 pi/3, the smallest, which is
// minus the largest root for -r).  The FP32 estimate 2 cos_acos3 is within
// ~2e-7; one FP64 Halley step (cubic convergence) leaves < 1e-20 where the
// roots are well separated and ~1e-15 at the edge of the nearly repeated band
// (|1 -+ r| < kNearRepeated, where the pair comes from deflation instead).
__host__ __device__ __forceinline__ double depressed_root(double r, bool largest)
{
    const double rr = largest ? r : -r;
    double x = 2.0 * (double)cos_acos3((float)(0.5 + 0.5 * rr));
    const double f = x * (x * x - 3.0) - 2.0 * rr;
    const double f1 = 3.0 * (x * x - 1.0);
    const double f2 = 6.0 * x;
    x -= (2.0 * f * f1) * rcp1(2.0 * f1 * f1 - f * f2);
    return largest ? x : -x;
}

// ---------------------------------------------------------------------------
// Eigenvalues.  With q = tr(H)/3, p = sqrt(tr((H - qI)^2)/6) and
// r = det((H - qI)/p)/2, the eigenvalues are q + 2p cos(phi + 2 pi k/3),
// phi = acos(r)/3, k = 0 giving the largest and k = 1 the smallest.
// ---------------------------------------------------------------------------
struct Hess64 {
    double xx, yy, zz, xy, xz, yz;
};

// q = tr/3, p and r of the trigonometric solution.  p == 0 (a multiple of
// the identity) gives r = 0 and every eigenvalue equal to q.  r -> -1 means
// l1 ~ l2 and r -> +1 means l2 ~ l3; near either end the cubic has a nearly
// double root and the pair loses about half its digits.
__host__ __device__ __forceinline__ void eig_moments(const Hess64& h, double& q, double& p, double& r)
{
    q = (h.xx + h.yy + h.zz) * (1.0 / 3.0);
    const double dx = h.xx - q, dy = h.yy - q, dz = h.zz - q;
    const double off = h.xy * h.xy + h.xz * h.xz + h.yz * h.yz;
    const double ss = dx * dx + dy * dy + dz * dz + 2.0 * off;
    // p and 1/p from one refined reciprocal square root; below the normal
    // range (no anisotropy to speak of) the matrix is taken as isotropic
    const double v = ss * (1.0 / 6.0);
    const bool iso = !(v >= 2.2250738585072014e-308);
    const double iv = rsq2(iso ? 1.0 : v);
    p = iso ? 0.0 : v * iv;
    const double ip = iso ? 0.0 : iv;
    const double det = dx * (dy * dz - h.yz * h.yz) - h.xy * (h.xy * dz - h.yz * h.xz) + h.xz * (h.xy * h.yz - dy * h.xz);
    r = 0.5 * det * (ip * ip * ip);
    r = fmin(fmax(r, -1.0), 1.0);
}

// Threshold on 1 -+ r below which the repeated pair is recomputed by
// deflation.  Above it the closed form keeps ~1e-12 relative accuracy.
constexpr double kNearRepeated = 1e-6;

// The two eigenvalues orthogonal to a well-separated eigenvalue mu: the
// eigenvector v of mu is the largest cross product of two rows of H - mu I;
// H projected on an orthonormal basis (u, w) of the plane normal to v is a
// 2x2 block whose eigenvalues m +- sqrt(((b11 - b22)/2)^2 + b12^2) have no
// cancellation however close they are.
__host__ __device__ __forceinline__ void deflate_pair(const Hess64& h, double mu, double& hi, double& lo)
{
    const double r0x = h.xx - mu, r0y = h.xy, r0z = h.xz;
    const double r1x = h.xy, r1y = h.yy - mu, r1z = h.yz;
    const double r2x = h.xz, r2y = h.yz, r2z = h.zz - mu;
    double ax = r0y * r1z - r0z * r1y, ay = r0z * r1x - r0x * r1z, az = r0x * r1y - r0y * r1x;
    const double bx = r0y * r2z - r0z * r2y, by = r0z * r2x - r0x * r2z, bz = r0x * r2y - r0y * r2x;
    const double cx = r1y * r2z - r1z * r2y, cy = r1z * r2x - r1x * r2z, cz = r1x * r2y - r1y * r2x;
    double na = ax * ax + ay * ay + az * az;
    const double nb = bx * bx + by * by + bz * bz;
    const double nc = cx * cx + cy * cy + cz * cz;
    if (nb > na) {
        ax = bx; ay = by; az = bz; na = nb;
    }
    if (nc > na) {
        ax = cx; ay = cy; az = cz; na = nc;
    }
    if (!(na > 0.0)) {
        hi = lo = mu;
        return;
    }
    const double iv = 1.0 / sqrt(na);
    const double vx = ax * iv, vy = ay * iv, vz = az * iv;
    // u: v crossed with the coordinate axis least aligned with v
    double ux, uy, uz;
    if (fabs(vx) <= fabs(vy) && fabs(vx) <= fabs(vz)) {
        ux = 0.0; uy = vz; uz = -vy;
    } else if (fabs(vy) <= fabs(vz)) {
        ux = -vz; uy = 0.0; uz = vx;
    } else {
        ux = vy; uy = -vx; uz = 0.0;
    }
    const double iu = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
    ux *= iu; uy *= iu; uz *= iu;
    const double wx = vy * uz - vz * uy, wy = vz * ux - vx * uz, wz = vx * uy - vy * ux;
    const double hux = h.xx * ux + h.xy * uy + h.xz * uz;
    const double huy = h.xy * ux + h.yy * uy + h.yz * uz;
    const double huz = h.xz * ux + h.yz * uy + h.zz * uz;
    const double hwx = h.xx * wx + h.xy * wy + h.xz * wz;
    const double hwy = h.xy * wx + h.yy * wy + h.yz * wz;
    const double hwz = h.xz * wx + h.yz * wy + h.zz * wz;
    const double b11 = ux * hux + uy * huy + uz * huz;
    const double b22 = wx * hwx + wy * hwy + wz * hwz;
    const double b12 = ux * hwx + uy * hwy + uz * hwz;
    const double m = 0.5 * (b11 + b22);
    const double d = sqrt(0.25 * (b11 - b22) * (b11 - b22) + b12 * b12);
    hi = m + d;
    lo = m - d;
}

// Largest eigenvalue l1 together with s = l2 + l3 and pp = l2 * l3, the only
// combinations the axis-1 collapse condition needs.  s = tr - l1 and
// pp = mu2 - l1 s, mu2 the sum of the principal 2x2 minors.
__host__ __device__ __forceinline__ void eig_top(const Hess64& h, double& l1, double& s, double& pp)
{
    double q, p, r;
    eig_moments(h, q, p, r);
    l1 = q + p * depressed_root(r, true);
    if (1.0 + r < kNearRepeated) {
        // l1 ~ l2: l3 (a simple root there) is well separated, the pair
        // comes from the 2x2 block
        double lo;
        const double l3 = q + p * depressed_root(r, false);
        deflate_pair(h, l3, l1, lo);
    }
    const double tr = h.xx + h.yy + h.zz;
    const double mu2 = h.xx * h.yy + h.xx * h.zz + h.yy * h.zz - h.xy * h.xy - h.xz * h.xz - h.yz * h.yz;
    s = tr - l1;
    pp = mu2 - l1 * s;
}

// All three eigenvalues, descending.
__host__ __device__ __forceinline__ void eig_all(const Hess64& h, double& l1, double& l2, double& l3)
{
    double q, p, r;
    eig_moments(h, q, p, r);
    // near either end of r one root of the depressed cubic is simple (well
    // conditioned) and the nearly repeated pair comes from deflation
    if (1.0 + r < kNearRepeated) {
        l3 = q + p * depressed_root(r, false);
        deflate_pair(h, l3, l1, l2);
    } else if (1.0 - r < kNearRepeated) {
        l1 = q + p * depressed_root(r, true);
        deflate_pair(h, l1, l2, l3);
    } else {
        l1 = q + p * depressed_root(r, true);
        l3 = q + p * depressed_root(r, false);
        l2 = (h.xx + h.yy + h.zz) - l1 - l3;
    }
    l2 = fmin(fmax(l2, l3), l1);
}

// ---------------------------------------------------------------------------
// Classic collapse.  Along the axis with eigenvalue l1 the LPT reading gives
//   R1/q1 = g(D) = 1 - l1 D + beta D^2 + gamma D^3,
//   beta  = -(3/14) l1 s,
//   gamma = -l1 [ (l1 s + 2 pp)/56 + 17 s^2/168 - pp/9 ],
// with s = l2 + l3 and pp = l2 l3.  D_c is its smallest positive root (the
// first crossing of the axis).  No root exists for l1 <= 0.  In u = l1 D:
//   g(u) = 1 - u + b u^2 + c u^3,  b = beta/l1^2,  c = gamma/l1^3.
// ---------------------------------------------------------------------------
struct CubicU {
    double b, c;
};

__host__ __device__ __forceinline__ double g_u(const CubicU& k, double u)
{
    return 1.0 + u * (-1.0 + u * (k.b + k.c * u));
}

__host__ __device__ __forceinline__ CubicU lpt_cubic(double l1, double s, double pp, double il1)
{
    const double sg = s * il1;
    const double pi = pp * (il1 * il1);
    CubicU k;
    k.b = (-3.0 / 14.0) * sg;
    k.c = -(sg * (1.0 / 56.0) + pi * (2.0 / 56.0) + (17.0 / 168.0) * (sg * sg) - pi * (1.0 / 9.0));
    return k;
}

// Bracket [lo, hi] on which g is monotone decreasing with g(lo) > 0 >= g(hi):
//  * the first positive critical point u1 = 1/(b + sqrt(b^2 + 3c)) is a local
//    minimum; if g(u1) <= 0 the root lies in (0, u1];
//  * if g(u1) > 0 and c >= 0, g rises for ever after u1: no root;
//  * if g(u1) > 0 and c < 0 the root lies past the local maximum
//    u2 = 1/(b - sqrt(b^2 + 3c));
//  * with no positive critical point g decreases on (0, inf).
// For c < 0, g(u) < 0 at u = max(1, 2 max(b, 0) / (-c)); for c = 0 without a
// critical point, b <= 0 and g(1) = b <= 0.
struct Bracket {
    double lo, hi;
    bool root;
};

__host__ __device__ __forceinline__ Bracket lpt_bracket(const CubicU& k)
{
    const double disc = k.b * k.b + 3.0 * k.c;
    const double sq = sqrt(fmax(disc, 0.0));
    const double den1 = k.b + sq;
    const bool has1 = disc >= 0.0 && den1 > 0.0;
    const double u1 = has1 ? rcp2(den1) : 0.0;
    const bool before_min = has1 && g_u(k, u1) <= 0.0;
    const double far = k.c < 0.0 ? fmax(1.0, 2.0 * fmax(k.b, 0.0) * rcp2(-k.c)) : 1.0;
    const bool past_max = has1 && !before_min && k.c < 0.0;
    Bracket br;
    br.root = !has1 || before_min || past_max;
    br.lo = past_max ? rcp2(k.b - sq) : 0.0;
    br.hi = before_min ? u1 : far;
    return br;
}

// FP32 estimate of the largest real root of w^3 - w^2 + b w + c, which is
// 1/u of the smallest positive root of g (w = 1/u maps one onto the other).
// Depressed with w = t + 1/3: t^3 + P t + Q = 0.  Three real roots: the
// largest is m cos(acos(3Q/(P m))/3), m = 2 sqrt(-P/3); one real root: the
// cancellation-free Cardano form A - P/(3A), A = -sign(Q) cbrt(|Q|/2 + sqrt(d)).
__host__ __device__ __forceinline__ float top_root_guess(double b, double c)
{
    const float P = (float)(b - 1.0 / 3.0);
    const float Q = (float)(c + b * (1.0 / 3.0) - 2.0 / 27.0);
    const float p3 = P * (1.0f / 3.0f);
    const float d = 0.25f * Q * Q + p3 * p3 * p3;
    float t;
    if (d <= 0.0f) {
        const float m = 2.0f * sqrtf(fmaxf(-p3, 0.0f));
        const float arg = fminf(fmaxf(3.0f * Q * __builtin_amdgcn_rcpf(P * m), -1.0f), 1.0f);
        t = m * cos_acos3(0.5f + 0.5f * arg);
    } else {
        // cube root from the hardware base-2 logarithm and exponential
        // (a few ulp; the FP64 polish that follows absorbs it)
        const float y = 0.5f * fabsf(Q) + sqrtf(d);
        const float A = -copysignf(__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(y) * (1.0f / 3.0f)), Q);
        t = A != 0.0f ? A - P * __builtin_amdgcn_rcpf(3.0f * A) : 0.0f;
    }
    return t + (1.0f / 3.0f);
}

// Halley iteration kept inside the bracket (bisection when a step leaves it);
// stops when the step is below a few ulps.  The start is the FP32 estimate
// above, so two steps normally reach full FP64 accuracy; the bracket makes the
// result the smallest positive root whatever the estimate.
__host__ __device__ __forceinline__ double lpt_solve_u(const CubicU& k, Bracket br)
{
    const float w0 = top_root_guess(k.b, k.c);
    double u = rcp2((double)w0);
    double lo = br.lo, hi = br.hi;
    if (!(u > lo && u < hi))
        u = 0.5 * (lo + hi);
    for (int it = 0; it < 80; ++it) {
        const double g = g_u(k, u);
        if (g == 0.0)
            break;  // landed on the root
        const double g1 = -1.0 + u * (2.0 * k.b + 3.0 * k.c * u);
        const double g2 = 2.0 * k.b + 6.0 * k.c * u;
        if (g > 0.0)
            lo = u;
        else
            hi = u;
        double un = u - (2.0 * g * g1) * rcp2(2.0 * g1 * g1 - g * g2);
        // inclusive: a step below one ulp leaves u on a bracket end
        if (!(un >= lo && un <= hi))
            un = 0.5 * (lo + hi);
        const double step = fabs(un - u);
        u = un;
        if (step <= 4e-16 * u)
            break;
    }
    return u;
}

// Direct solve in w = 1/u: the collapse is the largest real root of the monic
// cubic q(w) = w^3 - w^2 + b w + c (F = l1 w, no collapse when it is <= 0).
// Two FP64 Halley steps polish the FP32 estimate.  The result is accepted
// when the last step was small (converged) and w is provably the largest
// root: either q has no critical points (1 - 3b <= 0, q increasing), or w
// lies past the upper critical point wc = (1 + sqrt(1 - 3b))/3 (taken with a
// margin above the FP32 rounding of wc), or q's local minimum at wc is
// positive (one real root).  Otherwise the bracketed solver decides.
__host__ __device__ __forceinline__ bool top_root_w(const CubicU& k, double& w)
{
    w = (double)top_root_guess(k.b, k.c);
    double step = 0.0;
    for (int it = 0; it < 2; ++it) {
        const double q = ((w - 1.0) * w + k.b) * w + k.c;
        const double q1 = (3.0 * w - 2.0) * w + k.b;
        const double q2 = 6.0 * w - 2.0;
        step = (2.0 * q * q1) * rcp1(2.0 * q1 * q1 - q * q2);
        w -= step;
    }
    const bool converged = fabs(step) <= 1e-7 * fabs(w);
    const float e = (float)(1.0 - 3.0 * k.b);
    bool largest = true;
    if (e > 0.0f) {
        const double wc = (double)((1.0f + sqrtf(e)) * (1.0f / 3.0f));
        const double qc = ((wc - 1.0) * wc + k.b) * wc + k.c;
        largest = w >= wc * (1.0 + 1e-6) || qc > 0.0;
    }
    return converged && largest;
}

// F = 1/D_c, 0 without collapse.
__host__ __device__ __forceinline__ double classic_F(double l1, double s, double pp)
{
    if (!(l1 > 0.0))
        return 0.0;
    const double il1 = rcp2(l1);
    const CubicU k = lpt_cubic(l1, s, pp, il1);
    double w;
    if (!top_root_w(k, w)) {
        // nearly tangent or unconverged: bracketed solve in u = 1/w
        const Bracket br = lpt_bracket(k);
        w = br.root ? rcp2(lpt_solve_u(k, br)) : 0.0;
    }
    return w > 0.0 ? l1 * w : 0.0;
}

// ---------------------------------------------------------------------------
// Natural cubic spline evaluation on knots x[0..n-1] (LDS or global), values
// y and second derivatives m.  Interval i with x_i <= q < x_{i+1}; q at or past
// the last knot uses the last interval.  t = (q - x_i)/h:
//   S = (1-t) y_i + t y_{i+1} + h^2/6 [((1-t)^3 - (1-t)) m_i + (t^3 - t) m_{i+1}]
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int locate(const double* x, int n, double q)
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

__host__ __device__ __forceinline__ double spline_piece(double x0, double x1, double y0, double y1, double m0, double m1,
                                               double q)
{
    const double h = x1 - x0;
    const double t = (q - x0) * rcp2(h);
    const double w = 1.0 - t;
    return w * y0 + t * y1 + (h * h * (1.0 / 6.0)) * ((w * w * w - w) * m0 + (t * t * t - t) * m1);
}

// Interval lookup for the growth knots: bins uniform in log2(D) map a query
// to the first knot interval that can contain it (idx), and at most two
// compares finish the search; init verifies that bound for the table at hand
// (otherwise the plain binary search is used).  The interval found is the one
// `locate` finds.
struct GrowthIndex {
    const int* idx;  // nb entries (in LDS once staged)
    int nb;
    float L0;        // log2 of the first knot
    float S;         // bins per unit of log2 D
    int ok;          // the two-compare bound holds for this table
};

__host__ __device__ __forceinline__ int locate_indexed(const double* D, int n, double q, const GrowthIndex& gi)
{
    float fb = (__log2f((float)q) - gi.L0) * gi.S;
    fb = fminf(fmaxf(fb, 0.0f), (float)(gi.nb - 1));
    int i = gi.idx[(int)fb];
    i += (i + 1 <= n - 2 && D[i + 1] <= q) ? 1 : 0;
    i += (i + 1 <= n - 2 && D[i + 1] <= q) ? 1 : 0;
    return i;
}

// a(D) from the growth knots staged as [D | a | M] (n each).
__host__ __device__ __forceinline__ double growth_invert(const double* g, int n, double Dc, const GrowthIndex& gi)
{
    const double* D = g;
    const double* a = g + n;
    const double* M = g + 2 * n;
    if (!(Dc <= D[n - 1]))
        return kInf;
    if (Dc < D[0])
        return a[0];
    const int i = gi.ok ? locate_indexed(D, n, Dc, gi) : locate(D, n, Dc);
    return spline_piece(D[i], D[i + 1], a[i], a[i + 1], M[i], M[i + 1], Dc);
}

}  // namespace pino
