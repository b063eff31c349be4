// Classic collapse with the time coefficients of flat LCDM (Sec. 3: the LPT
// collapse condition; its second- and third-order terms grow, in LCDM, with
// growth functions of their own instead of the Einstein-de Sitter powers of
// D).
//
// Growth ratios.  With x = ln a, Om(a) = Om a^-3 / (Om a^-3 + 1 - Om) and
//   L[D] = D'' + (2 - 1.5 Om(a)) D' - 1.5 Om(a) D,
// the growing modes solve L[D1] = 0, L[D2] = -1.5 Om(a) D1^2,
// L[D3a] = -3 Om(a) D1^3 and L[D3b] = -3 Om(a) D1 (D2 - D1^2); in Einstein-de
// Sitter D2 = -(3/7) D1^2, D3a = -(1/3) D1^3, D3b = (10/21) D1^3.  The ratios
//   k2 = D2 / (-(3/7) D1^2), k3a = D3a / (-(1/3) D1^3), k3b = D3b / ((10/21) D1^3)
// scale the corresponding terms of the collapse condition.  k_lpt_growth
// integrates the eight first-order equations with classical RK4 in x, from
// the Einstein-de Sitter growing modes at a_s = 1e-7 a_0 (where the Lambda
// term is below 1e-20 of the matter term), in steps of at most 1e-3 that land
// on every knot of the growth table, and stores the ratios at the knots.
// The collapse kernels interpolate them with natural cubic splines in D over
// the same knots (held at the end values outside them).
//
// Collapse.  In u = l1 D the axis-1 condition becomes
//   G(u) = 1 - u + k2(D) b u^2 + (k3a(D) ca + k3b(D) cb) u^3,
// with b, ca + cb = c the Einstein-de Sitter coefficients of lpt_cubic split
// into the determinant-type part ca = pp / (9 l1^2) and the mixed part cb.
// The root: the Einstein-de Sitter cubic's first root u_e starts three
// Newton steps on G itself (ratio derivatives from the splines); the ratios
// move by about 1 % over the whole table, so u_e is that close to G's first
// root and the steps reach the rounding level.  Where they do not settle on a
// downward crossing near u_e, the cubic with the ratios frozen at D_e gives
// u1 (its first root, within ~1e-5 of G's) and two Newton steps finish it.
// The collapse kernels read the ratio splines in power form per interval
// (k_kappa_poly) where that fits in LDS, else as values and second
// derivatives at the knots; both describe the same cubic pieces.
#pragma once

#include "kernels_fp64.h"

namespace pino {

struct LptState {
    double d1, v1, d2, v2, d3a, v3a, d3b, v3b;
};

__device__ __forceinline__ LptState lpt_rhs(const LptState& y, double x, double om)
{
    const double a3 = exp(-3.0 * x);
    const double oma = om * a3 / (om * a3 + 1.0 - om);
    const double p = 2.0 - 1.5 * oma;
    LptState d;
    d.d1 = y.v1;
    d.v1 = -p * y.v1 + 1.5 * oma * y.d1;
    d.d2 = y.v2;
    d.v2 = -p * y.v2 + 1.5 * oma * y.d2 - 1.5 * oma * y.d1 * y.d1;
    d.d3a = y.v3a;
    d.v3a = -p * y.v3a + 1.5 * oma * y.d3a - 3.0 * oma * y.d1 * y.d1 * y.d1;
    d.d3b = y.v3b;
    d.v3b = -p * y.v3b + 1.5 * oma * y.d3b - 3.0 * oma * y.d1 * (y.d2 - y.d1 * y.d1);
    return d;
}

__device__ __forceinline__ LptState lpt_axpy(const LptState& y, double h, const LptState& k)
{
    return LptState{y.d1 + h * k.d1,   y.v1 + h * k.v1,   y.d2 + h * k.d2,   y.v2 + h * k.v2,
                    y.d3a + h * k.d3a, y.v3a + h * k.v3a, y.d3b + h * k.d3b, y.v3b + h * k.v3b};
}

__device__ __forceinline__ LptState lpt_rk4(const LptState& y, double x, double h, double om)
{
    const LptState k1 = lpt_rhs(y, x, om);
    const LptState k2 = lpt_rhs(lpt_axpy(y, 0.5 * h, k1), x + 0.5 * h, om);
    const LptState k3 = lpt_rhs(lpt_axpy(y, 0.5 * h, k2), x + 0.5 * h, om);
    const LptState k4 = lpt_rhs(lpt_axpy(y, h, k3), x + h, om);
    const double w = h * (1.0 / 6.0);
    LptState o;
    o.d1 = y.d1 + w * (k1.d1 + 2.0 * (k2.d1 + k3.d1) + k4.d1);
    o.v1 = y.v1 + w * (k1.v1 + 2.0 * (k2.v1 + k3.v1) + k4.v1);
    o.d2 = y.d2 + w * (k1.d2 + 2.0 * (k2.d2 + k3.d2) + k4.d2);
    o.v2 = y.v2 + w * (k1.v2 + 2.0 * (k2.v2 + k3.v2) + k4.v2);
    o.d3a = y.d3a + w * (k1.d3a + 2.0 * (k2.d3a + k3.d3a) + k4.d3a);
    o.v3a = y.v3a + w * (k1.v3a + 2.0 * (k2.v3a + k3.v3a) + k4.v3a);
    o.d3b = y.d3b + w * (k1.d3b + 2.0 * (k2.d3b + k3.d3b) + k4.d3b);
    o.v3b = y.v3b + w * (k1.v3b + 2.0 * (k2.v3b + k3.v3b) + k4.v3b);
    return o;
}

// One thread per cosmology c: growth knots at growth + c * 3 nk_max ([D | a |
// M], a from offset nk[c]), ratios written to kap + c * 6 nk_max as
// [k2 | k3a | k3b] (nk[c] each, contiguous; the spline second derivatives
// [m2 | m3a | m3b] follow, so the six rows of a cosmology are the 6 nk[c]
// doubles the collapse kernels stage).
constexpr double kLptStep = 1e-3;

__global__ void __launch_bounds__(64) k_lpt_growth(const double* __restrict__ growth, const int* __restrict__ nk,
                                                  const double* __restrict__ omega, int n_cosmo, int nk_max,
                                                  double* __restrict__ kap)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cosmo)
        return;
    const int n = nk[c];
    const double* ak = growth + (size_t)c * 3 * nk_max + n;
    double* out = kap + (size_t)c * 6 * nk_max;
    const double om = omega[c];
    const double as = 1e-7 * ak[0];
    LptState y{as, as, -(3.0 / 7.0) * as * as, -(6.0 / 7.0) * as * as, -(1.0 / 3.0) * as * as * as,
               -as * as * as, (10.0 / 21.0) * as * as * as, (10.0 / 7.0) * as * as * as};
    double x = log(as);
    for (int k = 0; k < n; ++k) {
        const double xe = log(ak[k]);
        const int m = max(1, (int)ceil((xe - x) / kLptStep));
        const double h = (xe - x) / m;
        const double x0 = x;
        for (int j = 0; j < m; ++j)
            y = lpt_rk4(y, x0 + h * j, h, om);
        x = xe;
        out[k] = y.d2 / (-(3.0 / 7.0) * y.d1 * y.d1);
        out[n + k] = y.d3a / (-(1.0 / 3.0) * y.d1 * y.d1 * y.d1);
        out[2 * n + k] = y.d3b / ((10.0 / 21.0) * y.d1 * y.d1 * y.d1);
    }
}

// LDS: the growth knots and index of stage_growth, then (from a 16-byte
// boundary) the ratio splines of the item's cosmology: the six rows
// [k2 | k3a | k3b | m2 | m3a | m3b] (nk each), or their power-form
// coefficients (kappa_poly_doubles(nk), k_kappa_poly).
__host__ __device__ inline size_t lcdm_table_offset(int nk, int nb)
{
    return (growth_lds_bytes(nk, nb) + 15) / 16 * 16;
}

__host__ __device__ inline size_t kappa_poly_doubles(int nk)
{
    return 12 * ((size_t)nk + 1);
}

__host__ __device__ inline size_t lcdm_lds_bytes(int nk, int nb)
{
    return lcdm_table_offset(nk, nb) + 6 * (size_t)nk * sizeof(double);
}

__host__ __device__ inline size_t lcdm_poly_lds_bytes(int nk, int nb)
{
    return lcdm_table_offset(nk, nb) + kappa_poly_doubles(nk) * sizeof(double);
}

// Power-form coefficients of the ratio splines, one thread per slot.  On
// [D_i, D_{i+1}], with h = D_{i+1} - D_i and s = D - D_i, the natural spline
// through (k_i, M_i) and (k_{i+1}, M_{i+1}) is
//   k_i + ((k_{i+1} - k_i)/h - h (2 M_i + M_{i+1})/6) s + (M_i/2) s^2
//       + ((M_{i+1} - M_i)/(6 h)) s^3.
// cf: slot i < n - 1 (interval i) at 12 i as [k2: c0 c1 c2 c3 | k3a: ... |
// k3b: ...]; slot n - 1 holds the constant piece at and above the last knot
// (c0 = the end value, c1 = c2 = c3 = 0), slot n the one at and below the
// first; kappa_poly_doubles(n) doubles.
__global__ void __launch_bounds__(256) k_kappa_poly(const double* __restrict__ D, const double* __restrict__ kap,
                                                   int n, double* __restrict__ cf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n)
        return;
    double* c = cf + 12 * i;
    if (i < n - 1) {
        const double h = D[i + 1] - D[i];
        for (int j = 0; j < 3; ++j) {
            const double k0 = kap[j * n + i], k1 = kap[j * n + i + 1];
            const double m0 = kap[(3 + j) * n + i], m1 = kap[(3 + j) * n + i + 1];
            c[4 * j] = k0;
            c[4 * j + 1] = (k1 - k0) / h - h * (2.0 * m0 + m1) / 6.0;
            c[4 * j + 2] = 0.5 * m0;
            c[4 * j + 3] = (m1 - m0) / (6.0 * h);
        }
    } else {
        const int e = i == n - 1 ? n - 1 : 0;
        for (int j = 0; j < 3; ++j) {
            c[4 * j] = kap[j * n + e];
            c[4 * j + 1] = c[4 * j + 2] = c[4 * j + 3] = 0.0;
        }
    }
}

// The three ratios and their derivatives in D.
struct Kappa {
    double k2, k3a, k3b, d2, d3a, d3b;
};

// One spline piece of the three ratios: interval [lo, hi) of the growth knots
// with the end values and second derivatives of each ratio, or (outside the
// knots, where the ratios are held at their end values) a constant piece.
// A Newton step whose D stays inside the piece reuses it from registers; the
// interval is the one the knot search returns for any D in (lo, hi), so the
// values are those of a fresh lookup.
struct KappaPiece {
    double lo, hi;
    double k2[2], k3a[2], k3b[2], m2[2], m3a[2], m3b[2];
    int kind;  // 0: interval of the knots, 1: below D_0 (or NaN), 2: at or above D_{n-1}
};

__device__ __forceinline__ bool piece_holds(const KappaPiece& p, double Dq)
{
    if (p.kind == 0)
        return Dq > p.lo && Dq < p.hi;
    return p.kind == 1 ? !(Dq > p.lo) : Dq >= p.hi;
}

// rows of kap: [k2 | k3a | k3b | m2 | m3a | m3b], nk each (LDS)
__device__ __forceinline__ KappaPiece kappa_piece(const double* D, const double* kap, int nk, double Dq,
                                                  const GrowthIndex& gi)
{
    KappaPiece p;
    if (!(Dq > D[0]) || !(Dq < D[nk - 1])) {
        const int e = Dq > D[0] ? nk - 1 : 0;
        p.kind = Dq > D[0] ? 2 : 1;
        p.lo = D[0];
        p.hi = D[nk - 1];
        p.k2[0] = p.k2[1] = kap[e];
        p.k3a[0] = p.k3a[1] = kap[nk + e];
        p.k3b[0] = p.k3b[1] = kap[2 * nk + e];
        p.m2[0] = p.m2[1] = p.m3a[0] = p.m3a[1] = p.m3b[0] = p.m3b[1] = 0.0;
        return p;
    }
    const int i = gi.ok ? locate_indexed(D, nk, Dq, gi) : locate(D, nk, Dq);
    p.kind = 0;
    p.lo = D[i];
    p.hi = D[i + 1];
    for (int j = 0; j < 2; ++j) {
        p.k2[j] = kap[i + j];
        p.k3a[j] = kap[nk + i + j];
        p.k3b[j] = kap[2 * nk + i + j];
        p.m2[j] = kap[3 * nk + i + j];
        p.m3a[j] = kap[4 * nk + i + j];
        p.m3b[j] = kap[5 * nk + i + j];
    }
    return p;
}

// the ratios and their derivatives at Dq from a piece that holds it
__device__ __forceinline__ Kappa kappa_eval(const KappaPiece& p, double Dq)
{
    Kappa r;
    if (p.kind != 0) {
        r.k2 = p.k2[0];
        r.k3a = p.k3a[0];
        r.k3b = p.k3b[0];
        r.d2 = r.d3a = r.d3b = 0.0;
        return r;
    }
    const double h = p.hi - p.lo;
    const double ih = rcp2(h);
    const double t = (Dq - p.lo) * ih;
    const double w = 1.0 - t;
    const double h6 = h * h * (1.0 / 6.0);
    const double cw = w * w * w - w, ct = t * t * t - t;
    const double dw = (h * (1.0 / 6.0)) * (1.0 - 3.0 * w * w), dt = (h * (1.0 / 6.0)) * (3.0 * t * t - 1.0);
    r.k2 = w * p.k2[0] + t * p.k2[1] + h6 * (cw * p.m2[0] + ct * p.m2[1]);
    r.k3a = w * p.k3a[0] + t * p.k3a[1] + h6 * (cw * p.m3a[0] + ct * p.m3a[1]);
    r.k3b = w * p.k3b[0] + t * p.k3b[1] + h6 * (cw * p.m3b[0] + ct * p.m3b[1]);
    r.d2 = (p.k2[1] - p.k2[0]) * ih + dw * p.m2[0] + dt * p.m2[1];
    r.d3a = (p.k3a[1] - p.k3a[0]) * ih + dw * p.m3a[0] + dt * p.m3a[1];
    r.d3b = (p.k3b[1] - p.k3b[0]) * ih + dw * p.m3b[0] + dt * p.m3b[1];
    return r;
}

// Where a solve reads the ratio splines.  KapRows: the six rows at the
// knots, a piece rebuilt from them at each lookup (the layout every table
// size fits).  KapPoly: the power-form coefficients of k_kappa_poly, so that
// a lookup reads one interval's 96 contiguous bytes and a step costs five
// FMAs per ratio.  D: the growth knots (D row); both in LDS or global memory.
struct KapRows {
    const double* D;
    const double* kap;
    int nk;
    GrowthIndex gi;
};

struct KapPoly {
    const double* D;
    const double* cf;  // 16-byte aligned
    int nk;
    GrowthIndex gi;
};

__device__ __forceinline__ KappaPiece piece_at(const KapRows& r, double Dq)
{
    return kappa_piece(r.D, r.kap, r.nk, Dq, r.gi);
}

// One slot of KapPoly: an interval (c[j] the coefficients of ratio j in
// s = D - lo) or a constant piece outside the knots (c[j][1..3] = 0), with
// the interval test of KappaPiece.
struct PolyPiece {
    double lo, hi;
    double c[3][4];
    int kind;  // as KappaPiece
};

__device__ __forceinline__ bool piece_holds(const PolyPiece& p, double Dq)
{
    if (p.kind == 0)
        return Dq > p.lo && Dq < p.hi;
    return p.kind == 1 ? !(Dq > p.lo) : Dq >= p.hi;
}

__device__ __forceinline__ PolyPiece piece_at(const KapPoly& r, double Dq)
{
    const double* D = r.D;
    const int nk = r.nk;
    PolyPiece p;
    int i;
    if (!(Dq > D[0]) || !(Dq < D[nk - 1])) {
        const bool above = Dq > D[0];
        p.kind = above ? 2 : 1;
        p.lo = D[0];
        p.hi = D[nk - 1];
        i = above ? nk - 1 : nk;
    } else {
        i = r.gi.ok ? locate_indexed(D, nk, Dq, r.gi) : locate(D, nk, Dq);
        p.kind = 0;
        p.lo = D[i];
        p.hi = D[i + 1];
    }
    // every slot is read the same way, so the coefficients need no merge
    // of two branches
    const d2v* q = reinterpret_cast<const d2v*>(r.cf + 12 * i);
    for (int j = 0; j < 3; ++j) {
        const d2v x = q[2 * j], y = q[2 * j + 1];
        p.c[j][0] = x.x;
        p.c[j][1] = x.y;
        p.c[j][2] = y.x;
        p.c[j][3] = y.y;
    }
    return p;
}

// the ratios and their derivatives at Dq: Horner's scheme, the derivative
// from the same partial sums (synthetic division)
__device__ __forceinline__ Kappa kappa_eval(const PolyPiece& p, double Dq)
{
    const double s = p.kind == 0 ? Dq - p.lo : 0.0;
    double v[3], d[3];
    for (int j = 0; j < 3; ++j) {
        const double b2 = fma(p.c[j][3], s, p.c[j][2]);
        const double b1 = fma(b2, s, p.c[j][1]);
        v[j] = fma(b1, s, p.c[j][0]);
        d[j] = fma(fma(p.c[j][3], s, b2), s, b1);
    }
    return Kappa{v[0], v[1], v[2], d[0], d[1], d[2]};
}

// w = 1/u of the first positive root of the cubic k (the Classic solver),
// <= 0 without one
__device__ __forceinline__ double cubic_top_w(const CubicU& k)
{
    double w;
    if (!top_root_w(k, w)) {
        const Bracket br = lpt_bracket(k);
        w = br.root ? rcp2(lpt_solve_u(k, br)) : 0.0;
    }
    return w;
}

// Start of the Newton steps on G: the first positive root w = 1/u_e of the
// Einstein-de Sitter cubic k to about 1e-5, which is all a start ~1 % from
// G's root needs: the FP32 estimate of top_root_w and one FP64 Halley step
// (top_root_w takes two, for a root to the rounding level), with its test
// that w is the cubic's largest root.  false if the step did not settle or
// the test fails.
__device__ __forceinline__ bool eds_start_w(const CubicU& k, double& w)
{
    w = (double)top_root_guess(k.b, k.c);
    const double q = ((w - 1.0) * w + k.b) * w + k.c;
    const double q1 = (3.0 * w - 2.0) * w + k.b;
    const double q2 = 6.0 * w - 2.0;
    const double step = (2.0 * q * q1) * rcp1(2.0 * q1 * q1 - q * q2);
    w -= step;
    bool ok = fabs(step) <= 1e-5 * fabs(w) && w > 0.0;
    const float e = (float)(1.0 - 3.0 * k.b);
    if (e > 0.0f) {
        const double wc = (double)((1.0f + sqrtf(e)) * (1.0f / 3.0f));
        const double qc = ((wc - 1.0) * wc + k.b) * wc + k.c;
        ok = ok && (w >= wc * (1.0 + 1e-6) || qc > 0.0);
    }
    return ok;
}

// Newton steps on G.  From the Einstein-de Sitter root (within the LCDM
// correction, under 1 %, of G's root) three steps reach the rounding level;
// from the frozen-ratio root (within about 1e-5) two do (a third moves D_c by
// under 1e-15 relative over 256^3 particles x 25 radii).
constexpr int kLcdmNewtonFromEds = 3;
constexpr int kLcdmNewton = 2;

// n Newton steps on G from u; returns false if the last step still moved u
// by more than 1e-7 of it (with quadratic convergence the error left after
// a step of 1e-7 is of order 1e-14 times G''/G' u), or G does not cross
// downward there (the first root of G, which starts at G(0) = 1, is a
// downward crossing).
template <class Src>
__device__ __forceinline__ bool lcdm_newton(double& u, int n, double il1, double b, double ca, double cb,
                                            const Src& src)
{
    auto pc = piece_at(src, u * il1);
    double du = 0.0, dG = -1.0;
    for (int it = 0; it < n; ++it) {
        const double Dq = u * il1;
        if (!piece_holds(pc, Dq))
            pc = piece_at(src, Dq);
        const Kappa k = kappa_eval(pc, Dq);
        const double P = k.k2 * b;
        const double Q = k.k3a * ca + k.k3b * cb;
        const double G = 1.0 + u * (-1.0 + u * (P + Q * u));
        dG = -1.0 + u * (2.0 * P + 3.0 * Q * u) + (u * u) * il1 * (k.d2 * b + u * (k.d3a * ca + k.d3b * cb));
        du = G * rcp2(dG);
        u -= du;
    }
    return fabs(du) <= 1e-7 * fabs(u) && dG < 0.0;
}

// F = 1/D_c with the LCDM coefficients, 0 without collapse; src: the growth
// knots and ratio splines (KapRows or KapPoly).
//
// Fast path: Newton on G from the first root u_e of the Einstein-de Sitter
// cubic (eds_start_w), accepted when it converged to a downward crossing
// within 5 % of u_e (the ratios move by about 1 % over the table, so G's
// first root is that close to u_e unless G is nearly tangent there).
// Otherwise (or with no EdS root) the robust path: the EdS root to the
// rounding level, then the cubic with the ratios frozen at D_e (or at the
// last knot) gives the first root of a cubic within about 1e-5 of G, then
// Newton steps.
template <class Src>
__device__ __forceinline__ double lcdm_F(double l1, double s, double pp, const Src& src)
{
    if (!(l1 > 0.0))
        return 0.0;
    const double il1 = rcp2(l1);
    const double sg = s * il1;
    const double pi = pp * (il1 * il1);
    const double b = (-3.0 / 14.0) * sg;
    const double ca = pi * (1.0 / 9.0);
    const double cb = -(sg * (1.0 / 56.0) + pi * (2.0 / 56.0) + (17.0 / 168.0) * (sg * sg));
    double w;
    if (eds_start_w(CubicU{b, ca + cb}, w)) {
        const double ue = rcp2(w);
        double u = ue;
        if (lcdm_newton(u, kLcdmNewtonFromEds, il1, b, ca, cb, src) && fabs(u - ue) <= 0.05 * ue)
            return l1 * rcp2(u);
    }
    w = cubic_top_w(CubicU{b, ca + cb});
    const double De = w > 0.0 ? rcp2(l1 * w) : src.D[src.nk - 1];
    const Kappa k = kappa_eval(piece_at(src, De), De);
    w = cubic_top_w(CubicU{k.k2 * b, k.k3a * ca + k.k3b * cb});
    if (!(w > 0.0))
        return 0.0;
    double u = rcp2(w);
    lcdm_newton(u, kLcdmNewton, il1, b, ca, cb, src);
    return u > 0.0 ? l1 * rcp2(u) : 0.0;
}

// Per-radius kernels of the LCDM method, with the update of update_max.
// Blocks of up to 512 lanes: the LDS a block stages (about 70 KB with the
// power-form coefficients of 512 knots) allows two blocks per CU, as many
// as the registers do.  POLY: the ratios from the power-form coefficients
// (kap_all: kappa_poly_doubles(nk) doubles), else from the six rows.
template <bool POLY>
struct KapSrc {
    using type = KapRows;
};
template <>
struct KapSrc<true> {
    using type = KapPoly;
};

template <class Src>
__device__ __forceinline__ double lcdm_of(const Hess64& h, const Src& src)
{
    double l1, s, pp;
    eig_top(h, l1, s, pp);
    return lcdm_F(l1, s, pp, src);
}

// One particle per lane over a grid-stride loop (arrays not 16-byte
// aligned), the next element's loads issued before the current element's
// arithmetic.
template <bool POLY>
__global__ void __launch_bounds__(512) k_classic_lcdm_1(ItemArgs a, const double* __restrict__ kap_all)
{
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const GrowthIndex gi = stage_growth(lds, a);
    double* kap = lds + lcdm_table_offset(a.nk, a.gi.nb) / sizeof(double);
    stage(kap, kap_all, POLY ? (int)kappa_poly_doubles(a.nk) : 6 * a.nk);
    __syncthreads();
    const typename KapSrc<POLY>::type src{lds, kap, (int)a.nk, gi};
    const uint32_t n = (uint32_t)a.n;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    Hess64 hn{};
    double fn = 0.0;
    if (i < n) {
        hn = load_h64(a, i);
        fn = a.reset ? 0.0 : *elem(a.Fmax, i);
    }
    for (; i < n; i += stride) {
        const Hess64 h = hn;
        const double fm = fn;
        const uint32_t next = i + stride;
        if (next < n) {
            hn = load_h64(a, next);
            fn = a.reset ? 0.0 : *elem(a.Fmax, next);
        }
        update_max(a, lds, gi, i, lcdm_of(h, src), fm);
    }
}

// Two adjacent particles per lane, as k_classic_f64: two independent root
// solves per lane, whose dependent FP64 chains the scheduler interleaves,
// and whole-line paired loads and stores.  Alignment as k_classic_f64 (host
// check); an odd last element is done by one lane at the end.
template <bool POLY>
__global__ void __launch_bounds__(512) k_classic_lcdm(ItemArgs a, const double* __restrict__ kap_all)
{
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const GrowthIndex gi = stage_growth(lds, a);
    double* kap = lds + lcdm_table_offset(a.nk, a.gi.nb) / sizeof(double);
    stage(kap, kap_all, POLY ? (int)kappa_poly_doubles(a.nk) : 6 * a.nk);
    __syncthreads();
    const typename KapSrc<POLY>::type src{lds, kap, (int)a.nk, gi};
    const uint32_t n = (uint32_t)a.n;
    const uint32_t np = n / 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    Hess2 hn{};
    d2v fn{0.0, 0.0};
    if (p < np) {
        hn = load_h2(a, p);
        if (!a.reset)
            fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * p));
    }
    for (; p < np; p += stride) {
        const Hess2 h = hn;
        const d2v fm = fn;
        const uint32_t next = p + stride;
        if (next < np) {
            hn = load_h2(a, next);
            if (!a.reset)
                fn = *reinterpret_cast<const d2v*>(elem(a.Fmax, 2 * next));
        }
        const double F0 = lcdm_of(Hess64{h.xx.x, h.yy.x, h.zz.x, h.xy.x, h.xz.x, h.yz.x}, src);
        const double F1 = lcdm_of(Hess64{h.xx.y, h.yy.y, h.zz.y, h.xy.y, h.xz.y, h.yz.y}, src);
        update_pair(a, lds, gi, p, F0, F1, fm);
    }
    if ((n & 1u) && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t i = n - 1;
        const double fm = a.reset ? 0.0 : *elem(a.Fmax, i);
        update_max(a, lds, gi, i, lcdm_of(load_h64(a, i), src), fm);
    }
}

}  // namespace pino
