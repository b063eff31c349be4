// The homogeneous-ellipsoid collapse that fills the Tabulated table (Sec. 3:
// nine ODEs integrated with fourth-order Runge-Kutta until the density
// diverges, tabulated over delta, x, y).
//
// Model (the form of Bond & Myers 1996, with the external tide of linear
// theory), in units H0 = 1 and time t, for the semi-axes R_i of a unit
// Lagrangian sphere in flat LCDM (Om, 1 - Om):
//   d2R_i/dt2 = -(3/2) Om a^-3 R_i [1/3 + alpha_i delta / 2 + (D/D1)(l_i - (l1+l2+l3)/3)]
//               + (1 - Om) R_i,
// with 1 + delta = a^3/(R1 R2 R3); the bracket is the background's 1/3 plus
// the ellipsoid's uniform excess and its internal tide,
// (1 + delta)/3 + (alpha_i - 2/3) delta/2 = 1/3 + alpha_i delta/2, and
//   alpha_i = |x1 x2 x3| int_0^inf dtau / ((x_i^2 + tau)^(3/2) sqrt((x_j^2 + tau)(x_k^2 + tau)))
//           = (2/3) |x1 x2 x3| R_D(x_j^2, x_k^2, x_i^2),   x = R/a,  sum alpha = 2,
// Carlson's symmetric integral R_D evaluated by its duplication theorem and
// the terminating series of Carlson (1995) (DLMF 19.36.2).  D is the linear
// growing mode and D1 its value at a = 1 (the eigenvalues are linear
// quantities of today).
//
// Modified-gravity option: the gravity of the density perturbations (the
// ellipsoid's excess, its internal tide and the external tide, and the
// linear growth) is scaled by mu(a) = 1 + mu0 / E(a)^2, which in flat LCDM
// is 1 + mu0 Omega_L(a)/Omega_L: standard at early times, departing as the
// cosmological constant takes over.  The background is unchanged.  mu0 = 0
// is general relativity (the scaling is then an exact multiplication by 1).
//
// The axes are carried as their displacement from the unperturbed sphere,
// psi_i = R_i - a (early on a perturbation of 1e-7 would drown in the
// rounding of R itself); the background's own acceleration cancels and
//   d2psi_i/dt2 = ((1 - Om) - (1/2) Om a^-3) psi_i
//                 - (3/2) Om a^-3 R_i [alpha_i delta / 2 + (D/D1)(l_i - (l1+l2+l3)/3)].
// With da/dt = a E(a), E^2 = Om a^-3 + 1 - Om, and the linear growth
// dD/dt = Dd, dDd/dt = -2 E Dd + (3/2) Om a^-3 D, these are nine first-order
// equations (psi, dpsi/dt for three axes; a; D, Dd).
//
// Start at a_i = 1e-7 in the Zel'dovich growing mode: D = a,
// psi_i = -l_i a^2/D1, dpsi_i/dt = -2 l_i a^2 E/D1.  Steps: dt = h/E(a) (h in
// ln a), shortened to kappa sqrt(R/|d2R/dt2|) of the smallest axis near
// collapse (its own time scale: finite at a regular crossing, ~ (t_c - t)
// in a nearly spherical free fall).  Collapse: a step that takes an axis to
// R <= 0 is shortened to land on the crossing (regula falsi in the step
// length); an axis whose remaining time R/|dR/dt| falls below 1e-12 of a
// Hubble time is taken as collapsed where it is.  F = D1/D at collapse; no
// collapse by a_stop gives F = 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace pino {

constexpr double kEllAi = 1e-7;      // initial scale factor
constexpr double kEllAstop = 10.0;   // no collapse by then: F = 0
constexpr double kEllStep = 1e-2;    // RK4 step in ln a
constexpr double kEllKappa = 0.05;   // step limit near collapse, in units of sqrt(R/|d2R/dt2|)
constexpr int kEllMaxSteps = 1 << 20;

// Carlson's R_D(x, y, z) = (3/2) int_0^inf dt / ((t + z)^(3/2) sqrt((t + x)(t + y))),
// x, y >= 0 (not both 0), z > 0.  Each duplication step adds
// 3 * 4^-k / (sqrt(z)(z + lam)) and moves the arguments together by a factor
// of four; once their relative spread is below 3e-3 the degree-5 series in
// the spread (error ~ spread^6) finishes.
__host__ __device__ inline double carlson_rd(double x, double y, double z)
{
    double sum = 0.0, fac = 1.0;
    double mu = 0.2 * (x + y + 3.0 * z);
    double X = 0.0, Y = 0.0, Z = 0.0;
    for (int it = 0; it < 60; ++it) {
        const double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        const double lam = sx * sy + sy * sz + sz * sx;
        sum += fac / (sz * (z + lam));
        fac *= 0.25;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
        mu = 0.2 * (x + y + 3.0 * z);
        const double im = 1.0 / mu;
        X = (mu - x) * im;
        Y = (mu - y) * im;
        Z = (mu - z) * im;
        if (fmax(fabs(X), fmax(fabs(Y), fabs(Z))) < 3e-3)
            break;
    }
    const double E2 = X * Y - 6.0 * Z * Z;
    const double E3 = (3.0 * X * Y - 8.0 * Z * Z) * Z;
    const double E4 = 3.0 * (X * Y - Z * Z) * Z * Z;
    const double E5 = X * Y * Z * Z * Z;
    const double ser = 1.0 - (3.0 / 14.0) * E2 + (1.0 / 6.0) * E3 + (9.0 / 88.0) * E2 * E2 - (3.0 / 22.0) * E4 -
                       (9.0 / 52.0) * E2 * E3 + (3.0 / 26.0) * E5;
    return 3.0 * sum + fac * ser / (mu * sqrt(mu));
}

struct EllState {
    double P[3], W[3], a, D, Dd;  // psi_i = R_i - a, W_i = dpsi_i/dt
};

struct EllPar {
    double om, ol, mu0, D1, lext[3];
};

// The right-hand side.  Axis 0 has the largest eigenvalue and is the first
// to collapse: alpha_1 and alpha_2 come from R_D (they vanish with x_0,
// where delta diverges, and their product with delta stays finite), alpha_0
// = 2 - alpha_1 - alpha_2 (near 2 there, with no cancellation).  delta is
// formed from e_i = psi_i/a as -(sum of the products of the e_i)/vol, free
// of the cancellation of 1/vol - 1 while the e_i are small.
__host__ __device__ inline EllState ell_rhs(const EllState& y, const EllPar& P)
{
    const double ia = 1.0 / y.a;
    const double ia3 = ia * ia * ia;
    const double E = sqrt(P.om * ia3 + P.ol);
    const double e0 = y.P[0] * ia, e1 = y.P[1] * ia, e2 = y.P[2] * ia;
    const double x0 = 1.0 + e0, x1 = 1.0 + e1, x2 = 1.0 + e2;
    const double vol = x0 * x1 * x2;
    const double vm1 = (e0 + e1 + e2) + (e0 * e1 + e0 * e2 + e1 * e2) + e0 * e1 * e2;  // vol - 1
    const double delta = -vm1 / vol;
    const double q0 = x0 * x0, q1 = x1 * x1, q2 = x2 * x2;
    const double av = (2.0 / 3.0) * fabs(vol);
    double al[3];
    al[1] = av * carlson_rd(q0, q2, q1);
    al[2] = av * carlson_rd(q0, q1, q2);
    al[0] = 2.0 - al[1] - al[2];
    const double g = 1.5 * P.om * ia3;
    const double lin = P.ol - g * (1.0 / 3.0);
    const double dn = y.D / P.D1;
    // the perturbations' gravity, scaled by mu = 1 + mu0 / E^2 (exactly g
    // when mu0 = 0); the background term lin is unchanged
    const double gm = g * (1.0 + P.mu0 / (E * E));
    EllState d;
    for (int i = 0; i < 3; ++i) {
        const double R = y.a + y.P[i];
        d.P[i] = y.W[i];
        d.W[i] = lin * y.P[i] - gm * R * (0.5 * al[i] * delta + dn * P.lext[i]);
    }
    d.a = y.a * E;
    d.D = y.Dd;
    d.Dd = -2.0 * E * y.Dd + gm * y.D;
    return d;
}

__host__ __device__ inline EllState ell_axpy(const EllState& y, double h, const EllState& k)
{
    EllState o;
    for (int i = 0; i < 3; ++i) {
        o.P[i] = y.P[i] + h * k.P[i];
        o.W[i] = y.W[i] + h * k.W[i];
    }
    o.a = y.a + h * k.a;
    o.D = y.D + h * k.D;
    o.Dd = y.Dd + h * k.Dd;
    return o;
}

// one classical RK4 step of length h from y, whose derivative k1 is given
__host__ __device__ inline EllState ell_rk4(const EllState& y, const EllState& k1, double h, const EllPar& P)
{
    const EllState k2 = ell_rhs(ell_axpy(y, 0.5 * h, k1), P);
    const EllState k3 = ell_rhs(ell_axpy(y, 0.5 * h, k2), P);
    const EllState k4 = ell_rhs(ell_axpy(y, h, k3), P);
    const double w = h * (1.0 / 6.0);
    EllState o;
    for (int i = 0; i < 3; ++i) {
        o.P[i] = y.P[i] + w * (k1.P[i] + 2.0 * (k2.P[i] + k3.P[i]) + k4.P[i]);
        o.W[i] = y.W[i] + w * (k1.W[i] + 2.0 * (k2.W[i] + k3.W[i]) + k4.W[i]);
    }
    o.a = y.a + w * (k1.a + 2.0 * (k2.a + k3.a) + k4.a);
    o.D = y.D + w * (k1.D + 2.0 * (k2.D + k3.D) + k4.D);
    o.Dd = y.Dd + w * (k1.Dd + 2.0 * (k2.Dd + k3.Dd) + k4.Dd);
    return o;
}

// the smallest semi-axis R_i = a + psi_i
__host__ __device__ inline double ell_rmin(const EllState& y)
{
    return y.a + fmin(y.P[0], fmin(y.P[1], y.P[2]));
}

// D(a = 1) of the growing mode started as D = a at a_i: RK4 in s = ln a of
// D'' = -(2 - 1.5 Om(a)) D' + 1.5 Om(a) mu(a) D in steps of 1e-4 (host side,
// at the call; it only normalises D)
inline double ell_growth_today(double om, double mu0)
{
    const double s0 = std::log(kEllAi);
    const int n = (int)std::ceil(-s0 / 1e-4);
    const double h = -s0 / n;
    double d = kEllAi, v = kEllAi;
    auto f = [om, mu0](double s, double dd, double vv, double& kd, double& kv) {
        const double a3 = std::exp(-3.0 * s);
        const double e2 = om * a3 + 1.0 - om;
        const double oma = om * a3 / e2;
        kd = vv;
        kv = -(2.0 - 1.5 * oma) * vv + 1.5 * oma * (1.0 + mu0 / e2) * dd;
    };
    for (int m = 0; m < n; ++m) {
        const double s = s0 + m * h;
        double k1d, k1v, k2d, k2v, k3d, k3v, k4d, k4v;
        f(s, d, v, k1d, k1v);
        f(s + 0.5 * h, d + 0.5 * h * k1d, v + 0.5 * h * k1v, k2d, k2v);
        f(s + 0.5 * h, d + 0.5 * h * k2d, v + 0.5 * h * k2v, k3d, k3v);
        f(s + h, d + h * k3d, v + h * k3v, k4d, k4v);
        d += h / 6.0 * (k1d + 2.0 * (k2d + k3d) + k4d);
        v += h / 6.0 * (k1v + 2.0 * (k2v + k3v) + k4v);
    }
    return d;
}

// F = 1/D_c of the ellipsoid with eigenvalues l0 >= l1 >= l2, or 0; mu0:
// the modified-gravity option (0: general relativity), D1 its growth today.
__host__ __device__ inline double ellipsoid_F(double l0, double l1, double l2, double om, double mu0, double D1)
{
    EllPar P;
    P.om = om;
    P.ol = 1.0 - om;
    P.mu0 = mu0;
    P.D1 = D1;
    const double third = (l0 + l1 + l2) * (1.0 / 3.0);
    P.lext[0] = l0 - third;
    P.lext[1] = l1 - third;
    P.lext[2] = l2 - third;
    const double ai = kEllAi;
    const double Ei = sqrt(om / (ai * ai * ai) + P.ol);
    const double lam[3] = {l0, l1, l2};
    EllState y;
    for (int i = 0; i < 3; ++i) {
        y.P[i] = -lam[i] * ai * ai / D1;
        y.W[i] = -2.0 * lam[i] * ai * ai * Ei / D1;
    }
    y.a = ai;
    y.D = ai;
    y.Dd = ai * Ei;
    for (int step = 0; step < kEllMaxSteps; ++step) {
        if (!(y.a < kEllAstop))
            return 0.0;
        const EllState k1 = ell_rhs(y, P);
        const double E = k1.a / y.a;
        int im = 0;
        if (y.P[1] < y.P[im])
            im = 1;
        if (y.P[2] < y.P[im])
            im = 2;
        const double R = y.a + y.P[im];
        const double V = k1.a + y.W[im];
        // an axis this close to zero, still falling, is collapsed
        if (V < 0.0 && R * E < -1e-12 * V)
            return D1 / y.D;
        double dt = kEllStep / E;
        const double acc = fabs(k1.W[im] + (P.ol - 0.5 * P.om / (y.a * y.a * y.a)) * y.a);  // d2R/dt2
        if (acc > 0.0)
            dt = fmin(dt, kEllKappa * sqrt(R / acc));
        EllState yn = ell_rk4(y, k1, dt, P);
        const double fn = ell_rmin(yn);
        if (!(fn > 0.0)) {
            // land on the crossing: regula falsi (Illinois) in the step
            // length on the smallest axis at the step's end
            double lo = 0.0, flo = R, hi = dt, fhi = fn;
            int side = 0;
            for (int it = 0; it < 60; ++it) {
                double tc = (lo * fhi - hi * flo) / (fhi - flo);
                if (!(tc > lo && tc < hi))
                    tc = 0.5 * (lo + hi);
                yn = ell_rk4(y, k1, tc, P);
                const double fc = ell_rmin(yn);
                if (fc > 0.0) {
                    lo = tc;
                    flo = fc;
                    if (side == 1)
                        fhi *= 0.5;
                    side = 1;
                } else {
                    hi = tc;
                    fhi = fc;
                    if (side == -1)
                        flo *= 0.5;
                    side = -1;
                }
                if (hi - lo <= 1e-15 * hi)
                    break;
            }
            yn = ell_rk4(y, k1, hi, P);
            return D1 / yn.D;
        }
        y = yn;
    }
    return 0.0;
}

// One thread per node of the (delta, x, y) table: knots dimensionless
// (xk[nx] | yk[ny] | dk[nd], scaled by sigma here), node (ix, iy, id) at
// thread (id * nx + ix) * ny + iy so that a wave holds nodes of one delta,
// out F[(ix * ny + iy) * nd + id].
__global__ void __launch_bounds__(256) k_ellipsoid_table(const double* __restrict__ knots, int nx, int ny, int nd,
                                                        double sigma, double om, double mu0, double D1,
                                                        double* __restrict__ F)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nodes = (int64_t)nx * ny * nd;
    if (t >= nodes)
        return;
    const int id = (int)(t / ((int64_t)nx * ny));
    const int r = (int)(t % ((int64_t)nx * ny));
    const int ix = r / ny, iy = r % ny;
    const double x = knots[ix] * sigma, yv = knots[nx + iy] * sigma, d = knots[nx + ny + id] * sigma;
    const double l0 = (d + 2.0 * x + yv) * (1.0 / 3.0);
    const double l1 = (d - x + yv) * (1.0 / 3.0);
    const double l2 = (d - x - 2.0 * yv) * (1.0 / 3.0);
    F[((int64_t)ix * ny + iy) * nd + id] = ellipsoid_F(l0, l1, l2, om, mu0, D1);
}

}  // namespace pino
