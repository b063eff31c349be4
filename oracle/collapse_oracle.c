/*
 * Oracle for the per-particle collapse-time computation.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 CPU implementation
 * written to be checked against the paper by eye.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the HIP
 * library never does, and the two share no source, header or table.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
 *
 * What it computes, with the passages it follows:
 *   - eigenvalues of the 3x3 Hessian of the smoothed potential, sorted in
 *     descending order (Sec. 3: "standard analytic method", sorted
 *     descending).  Here: cyclic Jacobi rotations, not the trigonometric
 *     closed form the kernel uses.
 *   - the Classic collapse: third-order LPT of a homogeneous ellipsoid gives a
 *     non-linear algebraic equation for the growth factor at collapse
 *     (Sec. 3).  The paper does not print the equation; the reading used is
 *     stated at orc_lpt_axis() below.  The smallest positive root is found by
 *     splitting (0, inf) at the critical points of the cubic and bisecting the
 *     first piece that changes sign.
 *   - the Tabulated collapse: a table over delta = sum l, x = l1 - l2,
 *     y = l2 - l3 interpolated with a cubic spline in delta and bilinearly in
 *     (x, y) (Sec. 3, Sec. 4.2).
 *   - the natural cubic spline (Sec. 4.2; the GSL routine the paper replaces
 *     is the natural spline) and the inversion of the growth table a(D)
 *     (Sec. 3, z_coll = 1/a_coll - 1).
 *   - the per-element maxima over smoothing radii (Sec. 4.1: the kernel
 *     updates two output arrays per element; here F = 1/D_c, its radius index,
 *     and a_coll).
 *   - D(a) of flat LCDM from the closed-form growth integral, used only to
 *     check the growth tables handed to both implementations.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CLASSIC 0
#define ORC_TABULATED 1

/* ------------------------------------------------------------------------ */
/* Eigenvalues: cyclic Jacobi on a symmetric 3x3 matrix.                    */
/* h = (xx, yy, zz, xy, xz, yz).  lam[0] >= lam[1] >= lam[2].               */
/* ------------------------------------------------------------------------ */
void orc_eig3(const double h[6], double lam[3])
{
    double A[3][3] = {{h[0], h[3], h[4]}, {h[3], h[1], h[5]}, {h[4], h[5], h[2]}};
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (!(off > 0.0) || off <= 1e-40 * dia)
            break;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[p][q];
                if (apq == 0.0)
                    continue;
                /* rotation angle that zeroes A[p][q] */
                double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150)
                    t = 0.5 / theta;
                else
                    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                A[p][p] -= t * apq;
                A[q][q] += t * apq;
                A[p][q] = A[q][p] = 0.0;
                for (int r = 0; r < 3; ++r) {
                    if (r == p || r == q)
                        continue;
                    double arp = A[r][p], arq = A[r][q];
                    A[r][p] = A[p][r] = c * arp - s * arq;
                    A[r][q] = A[q][r] = s * arp + c * arq;
                }
            }
        }
    }
    double d[3] = {A[0][0], A[1][1], A[2][2]};
    /* sort descending (three elements: plain exchange sort) */
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (d[j] > d[i]) {
                double tmp = d[i];
                d[i] = d[j];
                d[j] = tmp;
            }
    lam[0] = d[0];
    lam[1] = d[1];
    lam[2] = d[2];
}

/* ------------------------------------------------------------------------ */
/* Classic collapse: the LPT reading.                                       */
/*                                                                          */
/* Each principal axis of the Lagrangian sphere evolves as                  */
/*   R_i / q_i = 1 - l_i D + b_i D^2 + c_i D^3   (EdS growing modes),       */
/* where, with a_i = -l_i, A_i = sum_{j!=i} a_j, B_i = sum_{j!=i} b_j:      */
/*   b_i = -(3/14) l_i (l_1 + l_2 + l_3 - l_i)                              */
/*   c_i = -(1/12) a_i B_i - (17/36) b_i A_i - (1/9) a_1 a_2 a_3.           */
/* Their sums reproduce the second- and third-order LPT trace conditions    */
/* and, for l_1 = l_2 = l_3, the exact spherical-collapse series.  Collapse */
/* is the first crossing of the axis with the largest eigenvalue, R_1 = 0.  */
/* ------------------------------------------------------------------------ */
void orc_lpt_axis(const double lam[3], int axis, double *b_out, double *c_out)
{
    double a[3], b[3];
    double mu1 = lam[0] + lam[1] + lam[2];
    for (int i = 0; i < 3; ++i) {
        a[i] = -lam[i];
        b[i] = -(3.0 / 14.0) * lam[i] * (mu1 - lam[i]);
    }
    double A = 0.0, B = 0.0;
    for (int j = 0; j < 3; ++j) {
        if (j == axis)
            continue;
        A += a[j];
        B += b[j];
    }
    double c = -(1.0 / 12.0) * a[axis] * B - (17.0 / 36.0) * b[axis] * A - (1.0 / 9.0) * a[0] * a[1] * a[2];
    *b_out = b[axis];
    *c_out = c;
}

static double g_axis(double l1, double beta, double gamma, double D)
{
    return 1.0 - l1 * D + beta * D * D + gamma * D * D * D;
}

/* smallest positive root of g on (lo, hi], given g(lo) > 0 >= g(hi) and g
 * monotone on the piece: bisection down to adjacent doubles */
static double bisect(double l1, double beta, double gamma, double lo, double hi)
{
    for (int it = 0; it < 5000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi))
            break;
        if (g_axis(l1, beta, gamma, mid) > 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

/* Growth factor at collapse for sorted eigenvalues lam; *found = 0 when the
 * axis never collapses (returns 0). */
double orc_collapse_D(const double lam[3], int *found)
{
    double l1 = lam[0], beta, gamma;
    orc_lpt_axis(lam, 0, &beta, &gamma);
    *found = 0;
    if (!(isfinite(l1) && isfinite(beta) && isfinite(gamma)))
        return 0.0;

    /* positive critical points of g: roots of -l1 + 2 beta D + 3 gamma D^2 */
    double crit[2];
    int nc = 0;
    if (gamma == 0.0) {
        if (beta != 0.0) {
            double d = l1 / (2.0 * beta);
            if (d > 0.0)
                crit[nc++] = d;
        }
    } else {
        double disc = beta * beta + 3.0 * gamma * l1;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double Q = -(beta + (beta >= 0.0 ? sq : -sq));
            if (Q != 0.0) {
                double r1 = Q / (3.0 * gamma);
                double r2 = -l1 / Q;
                if (r1 > 0.0)
                    crit[nc++] = r1;
                if (r2 > 0.0)
                    crit[nc++] = r2;
                if (nc == 2 && crit[1] < crit[0]) {
                    double tmp = crit[0];
                    crit[0] = crit[1];
                    crit[1] = tmp;
                }
            }
        }
    }

    /* walk the monotone pieces [0, c1], [c1, c2], ... and bisect the first
     * one whose end values straddle zero */
    double lo = 0.0;
    for (int k = 0; k < nc; ++k) {
        double hi = crit[k];
        if (g_axis(l1, beta, gamma, lo) > 0.0 && g_axis(l1, beta, gamma, hi) <= 0.0) {
            *found = 1;
            return bisect(l1, beta, gamma, lo, hi);
        }
        lo = hi;
    }
    /* last piece [lo, inf): g goes to -inf only if its leading term is negative */
    int falls = (gamma < 0.0) || (gamma == 0.0 && beta < 0.0) || (gamma == 0.0 && beta == 0.0 && l1 > 0.0);
    if (!falls || !(g_axis(l1, beta, gamma, lo) > 0.0))
        return 0.0;
    double hi = lo > 0.0 ? 2.0 * lo : 1.0;
    while (g_axis(l1, beta, gamma, hi) > 0.0) {
        hi *= 2.0;
        if (hi > 1e300)
            return 0.0;
    }
    *found = 1;
    return bisect(l1, beta, gamma, lo, hi);
}

/* inverse collapse time F = 1/D_c, 0 when there is no collapse */
double orc_classic_F(const double lam[3])
{
    int found;
    double D = orc_collapse_D(lam, &found);
    return found ? 1.0 / D : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Natural cubic spline (second derivatives zero at both ends).             */
/* ------------------------------------------------------------------------ */

/* Second derivatives M[0..n-1].  Returns 0, or -1 if n < 2 or the knots are
 * not strictly increasing.  Tridiagonal system for the interior knots,
 *   h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
 *     = 6 [ (y_{i+1} - y_i)/h_i - (y_i - y_{i-1})/h_{i-1} ],
 * solved by Gaussian elimination without pivoting (diagonally dominant). */
int orc_spline_natural(int n, const double *x, const double *y, double *M)
{
    if (n < 2)
        return -1;
    for (int i = 0; i + 1 < n; ++i)
        if (!(x[i + 1] > x[i]))
            return -1;
    for (int i = 0; i < n; ++i)
        M[i] = 0.0;
    if (n == 2)
        return 0;
    int m = n - 2; /* unknowns M[1..n-2] */
    double *sub = (double *)malloc(sizeof(double) * m);
    double *dia = (double *)malloc(sizeof(double) * m);
    double *sup = (double *)malloc(sizeof(double) * m);
    double *rhs = (double *)malloc(sizeof(double) * m);
    for (int k = 0; k < m; ++k) {
        int i = k + 1;
        double hl = x[i] - x[i - 1], hr = x[i + 1] - x[i];
        sub[k] = hl;
        dia[k] = 2.0 * (hl + hr);
        sup[k] = hr;
        rhs[k] = 6.0 * ((y[i + 1] - y[i]) / hr - (y[i] - y[i - 1]) / hl);
    }
    /* forward elimination */
    for (int k = 1; k < m; ++k) {
        double f = sub[k] / dia[k - 1];
        dia[k] -= f * sup[k - 1];
        rhs[k] -= f * rhs[k - 1];
    }
    /* back substitution */
    M[m] = rhs[m - 1] / dia[m - 1];
    for (int k = m - 2; k >= 0; --k)
        M[k + 1] = (rhs[k] - sup[k] * M[k + 2]) / dia[k];
    free(sub);
    free(dia);
    free(sup);
    free(rhs);
    return 0;
}

/* index i with x[i] <= q < x[i+1]; q at or beyond the last knot maps to the
 * last interval, q below the first knot to the first */
static int locate(int n, const double *x, double q)
{
    int lo = 0, hi = n - 1;
    if (q >= x[n - 1])
        return n - 2;
    if (q <= x[0])
        return 0;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x[mid] <= q)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

/* S(q) on [x_i, x_{i+1}], t = (q - x_i)/h_i:
 *   S = (1-t) y_i + t y_{i+1} + (h_i^2/6) [((1-t)^3 - (1-t)) M_i + (t^3 - t) M_{i+1}] */
double orc_spline_eval(int n, const double *x, const double *y, const double *M, double q)
{
    int i = locate(n, x, q);
    double h = x[i + 1] - x[i];
    double t = (q - x[i]) / h;
    double s = 1.0 - t;
    return s * y[i] + t * y[i + 1] + (h * h / 6.0) * ((s * s * s - s) * M[i] + (t * t * t - t) * M[i + 1]);
}

/* a(D) through the natural spline of (D_k, a_k).  D beyond the last knot
 * (collapse after the end of the table) gives +inf; D below the first knot is
 * clamped to the first scale factor. */
double orc_growth_invert(int nk, const double *D, const double *a, const double *M, double Dc)
{
    if (!(Dc <= D[nk - 1]))
        return INFINITY;
    if (Dc < D[0])
        return a[0];
    return orc_spline_eval(nk, D, a, M, Dc);
}

/* ------------------------------------------------------------------------ */
/* Tabulated collapse: cubic spline in delta at the four corners of the     */
/* (x, y) cell, then bilinear interpolation.                                */
/* F[(ix*ny + iy)*nd + id], M the natural-spline second derivatives of each  */
/* delta row.  Out-of-range coordinates are clamped to the table.           */
/* ------------------------------------------------------------------------ */
double orc_table_F(int nx, int ny, int nd, const double *xk, const double *yk, const double *dk,
                   const double *F, const double *M, const double lam[3])
{
    double delta = lam[0] + lam[1] + lam[2];
    double x = lam[0] - lam[1];
    double y = lam[1] - lam[2];
    if (!(isfinite(delta) && isfinite(x) && isfinite(y)))
        return 0.0;
    int ix = locate(nx, xk, x);
    int iy = locate(ny, yk, y);
    double t = (x - xk[ix]) / (xk[ix + 1] - xk[ix]);
    double u = (y - yk[iy]) / (yk[iy + 1] - yk[iy]);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    double dq = delta;
    if (dq < dk[0]) dq = dk[0];
    if (dq > dk[nd - 1]) dq = dk[nd - 1];
    double v[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            size_t row = ((size_t)(ix + a) * ny + (iy + b)) * nd;
            v[a][b] = orc_spline_eval(nd, dk, F + row, M + row, dq);
        }
    double f = (1.0 - t) * (1.0 - u) * v[0][0] + t * (1.0 - u) * v[1][0] + (1.0 - t) * u * v[0][1] + t * u * v[1][1];
    return f > 0.0 ? f : 0.0;
}

/* second derivatives of every delta row of a table */
int orc_table_build(int nx, int ny, int nd, const double *dk, const double *F, double *M)
{
    for (int r = 0; r < nx * ny; ++r)
        if (orc_spline_natural(nd, dk, F + (size_t)r * nd, M + (size_t)r * nd) != 0)
            return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One smoothing radius: per particle, eigenvalues -> F -> max update.       */
/* ------------------------------------------------------------------------ */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count used by later parallel loops (n >= 1). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_update_radius(int64_t n, const double *hxx, const double *hyy, const double *hzz, const double *hxy,
                       const double *hxz, const double *hyz, int32_t radius_index, int method, int nk,
                       const double *gD, const double *ga, const double *gM, int nx, int ny, int nd,
                       const double *xk, const double *yk, const double *dk, const double *tF, const double *tM,
                       int reset, double *Fmax, int32_t *Rmax, double *acoll)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        if (reset) {
            Fmax[i] = 0.0;
            Rmax[i] = -1;
            if (acoll)
                acoll[i] = INFINITY;
        }
        double h[6] = {hxx[i], hyy[i], hzz[i], hxy[i], hxz[i], hyz[i]};
        double lam[3];
        orc_eig3(h, lam);
        double F, Dc;
        if (method == ORC_CLASSIC) {
            int found;
            Dc = orc_collapse_D(lam, &found);
            F = found ? 1.0 / Dc : 0.0;
        } else {
            F = orc_table_F(nx, ny, nd, xk, yk, dk, tF, tM, lam);
            Dc = 1.0 / F;
        }
        if (F > Fmax[i]) {
            Fmax[i] = F;
            Rmax[i] = radius_index;
            if (acoll)
                acoll[i] = orc_growth_invert(nk, gD, ga, gM, Dc);
        }
    }
}

/* per-point diagnostics: sorted eigenvalues and Classic F */
void orc_points(int64_t n, const double *h6, double *lam_out, double *F_out)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        double h[6];
        for (int c = 0; c < 6; ++c)
            h[c] = h6[(size_t)c * n + i];
        double lam[3];
        orc_eig3(h, lam);
        lam_out[3 * i + 0] = lam[0];
        lam_out[3 * i + 1] = lam[1];
        lam_out[3 * i + 2] = lam[2];
        F_out[i] = orc_classic_F(lam);
    }
}

/* ------------------------------------------------------------------------ */
/* Linear growth of flat LCDM from the closed-form integral                  */
/*   D(a) = (5 Om / 2) E(a) int_0^a da' / (a' E(a'))^3,                      */
/* substituting a' = t^2, which makes the integrand 2 t^4 (Om + OL t^6)^-3/2. */
/* Adaptive Simpson quadrature.                                             */
/* ------------------------------------------------------------------------ */
static double growth_integrand(double t, double om)
{
    double ol = 1.0 - om;
    double s = om + ol * t * t * t * t * t * t;
    return 2.0 * t * t * t * t / (s * sqrt(s));
}

static double simpson_rec(double a, double b, double fa, double fm, double fb, double whole, double tol, int depth,
                          double om)
{
    double m = 0.5 * (a + b);
    double lm = 0.5 * (a + m), rm = 0.5 * (m + b);
    double flm = growth_integrand(lm, om), frm = growth_integrand(rm, om);
    double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
    double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
    double delta = left + right - whole;
    if (depth <= 0 || fabs(delta) <= 15.0 * tol)
        return left + right + delta / 15.0;
    return simpson_rec(a, m, fa, flm, fm, left, 0.5 * tol, depth - 1, om) +
           simpson_rec(m, b, fm, frm, fb, right, 0.5 * tol, depth - 1, om);
}

double orc_growth_unnorm(double om, double a)
{
    double tb = sqrt(a);
    double fa = growth_integrand(0.0, om), fb = growth_integrand(tb, om), fm = growth_integrand(0.5 * tb, om);
    double whole = tb / 6.0 * (fa + 4.0 * fm + fb);
    double integral = simpson_rec(0.0, tb, fa, fm, fb, whole, 1e-14 * fabs(whole), 40, om);
    double E = sqrt(om / (a * a * a) + 1.0 - om);
    return 2.5 * om * E * integral;
}

double orc_growth_D(double om, double a)
{
    return orc_growth_unnorm(om, a) / orc_growth_unnorm(om, 1.0);
}

/* ------------------------------------------------------------------------ */
/* Higher-order LPT growth in flat LCDM (cosmology-dependent time           */
/* coefficients of the LPT collapse condition, Sec. 3).                      */
/*                                                                          */
/* With x = ln a, E^2 = Om a^-3 + 1 - Om and Om(a) = Om a^-3 / E^2, the     */
/* growing modes of the second and third LPT orders solve                    */
/*   L[D] = D'' + (2 - 1.5 Om(a)) D' - 1.5 Om(a) D                          */
/*   L[D1] = 0,  L[D2] = -1.5 Om(a) D1^2,  L[D3a] = -3 Om(a) D1^3,          */
/*   L[D3b] = -3 Om(a) D1 (D2 - D1^2),                                       */
/* which in Einstein-de Sitter give D2 = -(3/7) D1^2, D3a = -(1/3) D1^3 and  */
/* D3b = (10/21) D1^3.  Here they are NOT integrated as ODEs: the oracle     */
/* writes the solution by variation of parameters with the two homogeneous   */
/* solutions D+ = E I (the growing mode, I = (5 Om / 2) int_0^a da'/(a'E)^3) */
/* and D- = E (the decaying mode).  Their Wronskian is -(5 Om/2)/(a^2 E),    */
/* so a source f gives the growing-mode particular solution                  */
/*   D(a) = (2/(5 Om)) E(a) int_0^a [I(a) - I(a')] E(a')^2 a'^2 f(a') da'/a'. */
/* With the sources above this becomes                                       */
/*   D2  = -(3/5) E [I A2 - B2],  A2 = int D1^2 a^-2 da,  B2 = int I D1^2 a^-2 da, */
/*   D3a = -(6/5) E [I A3 - B3],  A3 = int D1^3 a^-2 da,  B3 = int I D1^3 a^-2 da, */
/*   D3b = -(6/5) E [I A4 - B4],  A4 = int D1 (D2 - D1^2) a^-2 da,  B4 likewise    */
/*   with a factor I,                                                           */
/* all integrals from 0.  Below a_s = 1e-7 a_0 (a_0 the first knot) the      */
/* Lambda term changes them by less than 1e-20 relative, so their values at  */
/* a_s are the Einstein-de Sitter power laws; from a_s on they are           */
/* accumulated by composite Simpson on a grid uniform in ln a, with every    */
/* knot a grid node and steps of at most 1e-3.  The outputs are the ratios   */
/* to the Einstein-de Sitter coefficients at each knot,                      */
/*   k2 = D2 / (-(3/7) D1^2),  k3a = D3a / (-(1/3) D1^3),                     */
/*   k3b = D3b / ((10/21) D1^3),                                              */
/* which do not depend on how D1 is normalised.                               */
/* ------------------------------------------------------------------------ */

/* cumulative integral over the nodes of one segment of uniform step h (m
 * steps, m even): S[0] = s0, then Simpson over node pairs for the even
 * nodes and, for the odd ones, the integral over one step of the quadratic
 * through that step's two nodes and the next, h/12 (5 f0 + 8 f1 - f2). */
static void cum_simpson(int m, double h, const double *f, double s0, double *S)
{
    S[0] = s0;
    for (int j = 0; j + 2 <= m; j += 2) {
        S[j + 1] = S[j] + h / 12.0 * (5.0 * f[j] + 8.0 * f[j + 1] - f[j + 2]);
        S[j + 2] = S[j] + h / 3.0 * (f[j] + 4.0 * f[j + 1] + f[j + 2]);
    }
}

int orc_lpt_growth(double om, int nk, const double *ak, double *k2, double *k3a, double *k3b)
{
    if (nk < 1 || !(om > 0.0) || !(ak[0] > 0.0))
        return -1;
    for (int k = 0; k + 1 < nk; ++k)
        if (!(ak[k + 1] > ak[k]))
            return -1;
    const double ol = 1.0 - om;
    /* segments: 0 over [a_s, a_0], k >= 1 over [a_{k-1}, a_k], each uniform
     * in ln a with an even number of steps of at most 1e-3 */
    const double as = 1e-7 * ak[0];
    int *ms = (int *)malloc(sizeof(int) * nk);
    double *hs = (double *)malloc(sizeof(double) * nk);
    int *st = (int *)malloc(sizeof(int) * nk);
    int total = 0, mmax = 0;
    for (int k = 0; k < nk; ++k) {
        double lo = (k == 0) ? as : ak[k - 1];
        double dx = log(ak[k] / lo);
        int m = (int)ceil(dx / 1e-3);
        if (m < 16)
            m = 16;
        m += m & 1;
        ms[k] = m;
        hs[k] = dx / m;
        st[k] = total;
        total += m;
        if (m > mmax)
            mmax = m;
    }
    const int nn = total + 1;
    double *a = (double *)malloc(sizeof(double) * nn);
    for (int k = 0; k < nk; ++k) {
        double x0 = log((k == 0) ? as : ak[k - 1]);
        if (k == 0)
            a[0] = as;
        for (int j = 1; j <= ms[k]; ++j)
            a[st[k] + j] = (j == ms[k]) ? ak[k] : exp(x0 + hs[k] * j);
    }
    double *E = (double *)malloc(sizeof(double) * nn);
    double *I = (double *)malloc(sizeof(double) * nn);
    double *r1 = (double *)malloc(sizeof(double) * nn); /* D1 / a */
    double *r2 = (double *)malloc(sizeof(double) * nn); /* D2 / a^2 */
    double *A = (double *)malloc(sizeof(double) * nn);
    double *B = (double *)malloc(sizeof(double) * nn);
    double *A3 = (double *)malloc(sizeof(double) * nn);
    double *B3 = (double *)malloc(sizeof(double) * nn);
    double *A4 = (double *)malloc(sizeof(double) * nn);
    double *B4 = (double *)malloc(sizeof(double) * nn);
    double *f = (double *)malloc(sizeof(double) * (mmax + 1));
    for (int j = 0; j < nn; ++j)
        E[j] = sqrt(om / (a[j] * a[j] * a[j]) + ol);

    /* OUT = s0 at a_s plus the cumulative integral of g da = g a dx, g the
     * expression gv of node q */
#define ACCUMULATE(gv, s0, OUT)                                                          \
    do {                                                                                 \
        double s = (s0);                                                                 \
        for (int k = 0; k < nk; ++k) {                                                   \
            for (int j = 0; j <= ms[k]; ++j) {                                           \
                int q = st[k] + j;                                                       \
                f[j] = (gv) * a[q];                                                      \
            }                                                                            \
            cum_simpson(ms[k], hs[k], f, s, OUT + st[k]);                                \
            s = OUT[st[k] + ms[k]];                                                      \
        }                                                                                \
    } while (0)

    /* Einstein-de Sitter values at a_s: I = a^(5/2)/sqrt(Om), D1 = a,
     * D2 = -(3/7) a^2 */
    const double sq = sqrt(om);
    const double i_s = as * as * sqrt(as) / sq;
    ACCUMULATE(2.5 * om / (a[q] * E[q] * a[q] * E[q] * a[q] * E[q]), i_s, I);
    for (int j = 0; j < nn; ++j)
        r1[j] = E[j] * I[j] / a[j];
    ACCUMULATE(r1[q] * r1[q], as, A);
    ACCUMULATE(I[q] * r1[q] * r1[q], (2.0 / 7.0) * i_s * as, B);
    for (int j = 0; j < nn; ++j)
        r2[j] = -0.6 * E[j] * (I[j] * A[j] - B[j]) / (a[j] * a[j]);
    ACCUMULATE(r1[q] * r1[q] * r1[q] * a[q], 0.5 * as * as, A3);
    ACCUMULATE(I[q] * r1[q] * r1[q] * r1[q] * a[q], (2.0 / 9.0) * i_s * as * as, B3);
    ACCUMULATE(r1[q] * (r2[q] - r1[q] * r1[q]) * a[q], -(5.0 / 7.0) * as * as, A4);
    ACCUMULATE(I[q] * r1[q] * (r2[q] - r1[q] * r1[q]) * a[q], -(10.0 / 7.0) * (2.0 / 9.0) * i_s * as * as, B4);
#undef ACCUMULATE
    for (int k = 0; k < nk; ++k) {
        int q = st[k] + ms[k];
        double d1 = r1[q] * a[q];
        double d2 = r2[q] * a[q] * a[q];
        double d3a = -1.2 * E[q] * (I[q] * A3[q] - B3[q]);
        double d3b = -1.2 * E[q] * (I[q] * A4[q] - B4[q]);
        k2[k] = d2 / (-(3.0 / 7.0) * d1 * d1);
        k3a[k] = d3a / (-(1.0 / 3.0) * d1 * d1 * d1);
        k3b[k] = d3b / ((10.0 / 21.0) * d1 * d1 * d1);
    }
    free(ms); free(hs); free(st); free(a); free(E); free(I); free(r1); free(r2);
    free(A); free(B); free(A3); free(B3); free(A4); free(B4); free(f);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Classic collapse with the LCDM time coefficients.  The EdS coefficients  */
/* of the axis-1 condition split as beta (second order), gamma_a (the        */
/* -(1/9) a1 a2 a3 part of c_1, a third-order term of determinant type) and  */
/* gamma_b = c_1 - gamma_a (the mixed first-times-second-order terms).  In   */
/* LCDM each is scaled by its growth ratio at the epoch where the growth     */
/* factor is D:                                                              */
/*   G(D) = 1 - l1 D + k2(D) beta D^2 + (k3a(D) gamma_a + k3b(D) gamma_b) D^3, */
/* with k2, k3a, k3b the natural cubic splines in D of their values at the   */
/* growth-table knots (D_k, from orc_lpt_growth at a_k), held at the end     */
/* values outside [D_0, D_{n-1}].  The collapse is the smallest positive     */
/* root of G: a sign scan on a geometric grid of 4001 points from 1e-4/L to  */
/* 1e4/L (L = max(|l1|, |l3|), ratio 1.0046), bisection of the first step    */
/* that reaches G <= 0, and past the grid the doubling search of the         */
/* constant-coefficient cubic.                                              */
/* ------------------------------------------------------------------------ */
static double kappa_at(int nk, const double *D, const double *k, const double *M, double Dq)
{
    if (Dq <= D[0])
        return k[0];
    if (Dq >= D[nk - 1])
        return k[nk - 1];
    return orc_spline_eval(nk, D, k, M, Dq);
}

typedef struct {
    int nk;
    const double *D, *k2, *m2, *k3a, *m3a, *k3b, *m3b;
} orc_kappa;

static double g_lcdm(const orc_kappa *K, double l1, double beta, double ga, double gb, double D)
{
    double k2 = kappa_at(K->nk, K->D, K->k2, K->m2, D);
    double k3a = kappa_at(K->nk, K->D, K->k3a, K->m3a, D);
    double k3b = kappa_at(K->nk, K->D, K->k3b, K->m3b, D);
    return 1.0 - l1 * D + k2 * beta * D * D + (k3a * ga + k3b * gb) * D * D * D;
}

static double bisect_lcdm(const orc_kappa *K, double l1, double beta, double ga, double gb, double lo, double hi)
{
    for (int it = 0; it < 5000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi))
            break;
        if (g_lcdm(K, l1, beta, ga, gb, mid) > 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

double orc_collapse_D_lcdm(const double lam[3], int nk, const double *D, const double *k2, const double *m2,
                           const double *k3a, const double *m3a, const double *k3b, const double *m3b, int *found)
{
    orc_kappa K = {nk, D, k2, m2, k3a, m3a, k3b, m3b};
    double l1 = lam[0], beta, c1;
    orc_lpt_axis(lam, 0, &beta, &c1);
    double ga = (1.0 / 9.0) * lam[0] * lam[1] * lam[2]; /* -(1/9) a1 a2 a3 with a_i = -l_i */
    double gb = c1 - ga;
    *found = 0;
    if (!(isfinite(l1) && isfinite(beta) && isfinite(c1)))
        return 0.0;
    double L = fabs(lam[0]) > fabs(lam[2]) ? fabs(lam[0]) : fabs(lam[2]);
    if (!(L > 0.0))
        return 0.0;
    const int npts = 4001;
    const double d0 = 1e-4 / L;
    const double ratio = pow(1e8, 1.0 / (npts - 1));
    double prev = 0.0, Dj = d0;
    for (int j = 0; j < npts; ++j) {
        if (g_lcdm(&K, l1, beta, ga, gb, Dj) <= 0.0) {
            *found = 1;
            return bisect_lcdm(&K, l1, beta, ga, gb, prev, Dj);
        }
        prev = Dj;
        Dj *= ratio;
    }
    /* past the grid (and past the last knot for any realistic L): the cubic
     * with the coefficients held at their last-knot values */
    double kb = k2[nk - 1] * beta, kc = k3a[nk - 1] * ga + k3b[nk - 1] * gb;
    int falls = (kc < 0.0) || (kc == 0.0 && kb < 0.0);
    if (!falls)
        return 0.0;
    double hi = 2.0 * prev;
    while (g_lcdm(&K, l1, beta, ga, gb, hi) > 0.0) {
        prev = hi;
        hi *= 2.0;
        if (hi > 1e300)
            return 0.0;
    }
    *found = 1;
    return bisect_lcdm(&K, l1, beta, ga, gb, prev, hi);
}

/* One smoothing radius of the Classic method with LCDM time coefficients
 * (same per-particle flow as orc_update_radius). */
void orc_update_radius_lcdm(int64_t n, const double *hxx, const double *hyy, const double *hzz, const double *hxy,
                            const double *hxz, const double *hyz, int32_t radius_index, int nk, const double *gD,
                            const double *ga, const double *gM, const double *k2, const double *m2,
                            const double *k3a, const double *m3a, const double *k3b, const double *m3b, int reset,
                            double *Fmax, int32_t *Rmax, double *acoll)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        if (reset) {
            Fmax[i] = 0.0;
            Rmax[i] = -1;
            if (acoll)
                acoll[i] = INFINITY;
        }
        double h[6] = {hxx[i], hyy[i], hzz[i], hxy[i], hxz[i], hyz[i]};
        double lam[3];
        orc_eig3(h, lam);
        int found;
        double Dc = orc_collapse_D_lcdm(lam, nk, gD, k2, m2, k3a, m3a, k3b, m3b, &found);
        double F = found ? 1.0 / Dc : 0.0;
        if (F > Fmax[i]) {
            Fmax[i] = F;
            Rmax[i] = radius_index;
            if (acoll)
                acoll[i] = orc_growth_invert(nk, gD, ga, gM, Dc);
        }
    }
}

/* G(D) of orc_collapse_D_lcdm and its derivative dG/dD by central
 * difference at step 1e-6 D (test diagnostics: near-tangent roots) */
double orc_g_lcdm(const double lam[3], int nk, const double *D, const double *k2, const double *m2,
                  const double *k3a, const double *m3a, const double *k3b, const double *m3b, double Dq,
                  double *dG)
{
    orc_kappa K = {nk, D, k2, m2, k3a, m3a, k3b, m3b};
    double beta, c1;
    orc_lpt_axis(lam, 0, &beta, &c1);
    double ga = (1.0 / 9.0) * lam[0] * lam[1] * lam[2];
    double gb = c1 - ga;
    if (dG) {
        double e = 1e-6 * Dq;
        *dG = (g_lcdm(&K, lam[0], beta, ga, gb, Dq + e) - g_lcdm(&K, lam[0], beta, ga, gb, Dq - e)) / (2.0 * e);
    }
    return g_lcdm(&K, lam[0], beta, ga, gb, Dq);
}

/* ------------------------------------------------------------------------ */
/* Homogeneous-ellipsoid collapse: the source of the Tabulated table         */
/* (Sec. 3: nine ODEs integrated with fourth-order Runge-Kutta until the     */
/* density diverges).  The equations are those of a homogeneous ellipsoid in */
/* an expanding flat LCDM background with the external tide of linear theory */
/* (the form of Bond & Myers 1996).  For semi-axes R_i = a x_i (unit          */
/* Lagrangian radius), with 1 + delta = 1/(x1 x2 x3):                         */
/*   d2R_i/dt2 = -(3/2) Om a^-3 R_i [1/3 + mu(a) (delta/3                    */
/*               + (alpha_i - 2/3) delta/2 + (D/D1) (l_i - (l1+l2+l3)/3))]    */
/*               + (1 - Om) R_i,                                             */
/*   alpha_i = |x1 x2 x3| int_0^inf dtau / ((x_i^2 + tau)^(3/2)              */
/*                                        sqrt((x_j^2 + tau)(x_k^2 + tau))), */
/* D the linear growing mode and D1 its value at a = 1.  mu(a) scales the     */
/* gravity of the density perturbations (the background is unchanged), a     */
/* modified-gravity option: mu = 1 + mu0 / E(a)^2 (in flat LCDM, 1 + mu0     */
/* Omega_L(a)/Omega_L), so gravity is standard at early times; mu0 = 0 is    */
/* general relativity.  The growth equation carries the same mu.              */
/*                                                                          */
/* The oracle does NOT integrate that form.  It integrates the equivalent     */
/* comoving system in s = ln a (eight ODEs; ' = d/ds, Om(a) = Om a^-3/E^2):   */
/*   x_i'' = -(2 - 1.5 Om(a)) x_i' - 1.5 Om(a) mu(a) x_i [delta/3             */
/*            + (alpha_i - 2/3) delta/2 + (D/D1)(l_i - (l1+l2+l3)/3)],        */
/*   D''   = -(2 - 1.5 Om(a)) D' + 1.5 Om(a) mu(a) D,                         */
/* with classical RK4 at a fixed step in s, alpha_i by the trapezoid rule in  */
/* v = ln tau (step 0.5 over the range where the integrand is above 1e-17 of  */
/* its scale; the integrand is analytic within |Im v| < pi, where this rule   */
/* converges geometrically, error ~ exp(-2 pi^2 / 0.5)), and the crossing of  */
/* x_1 = 0 located by bisection of the last step's length.  Initial state at  */
/* a_i: the Zel'dovich growing mode D = a, x_i = 1 - l_i a_i / D1.  No        */
/* collapse by a_stop gives F = 0.  Output F = 1/D_c, D_c = D(a_c)/D1.        */
/* ------------------------------------------------------------------------ */
static double ell_f(double v, double xi2, double xj2, double xk2)
{
    double t = exp(v);
    double u = xi2 + t;
    return t / (u * sqrt(u) * sqrt((xj2 + t) * (xk2 + t)));
}

/* alpha_i of axes x[0..2] */
double orc_ell_alpha(const double x[3], int i)
{
    int j = (i + 1) % 3, k = (i + 2) % 3;
    double xi2 = x[i] * x[i], xj2 = x[j] * x[j], xk2 = x[k] * x[k];
    double lo = xi2, hi = xi2;
    if (xj2 < lo) lo = xj2;
    if (xk2 < lo) lo = xk2;
    if (xj2 > hi) hi = xj2;
    if (xk2 > hi) hi = xk2;
    if (!(lo > 0.0))
        return (xi2 > 0.0) ? 0.0 : 2.0; /* a degenerate axis: the flat limits */
    const double h = 0.5;
    double v0 = log(lo) - 40.0, v1 = log(hi) + 28.0;
    int n = (int)ceil((v1 - v0) / h);
    double sum = 0.5 * (ell_f(v0, xi2, xj2, xk2) + ell_f(v0 + n * h, xi2, xj2, xk2));
    for (int m = 1; m < n; ++m)
        sum += ell_f(v0 + m * h, xi2, xj2, xk2);
    double I = h * sum;
    /* the part below v0, where the integrand is its tau -> 0 value times tau */
    I += exp(v0) / (xi2 * sqrt(xi2) * sqrt(xj2 * xk2));
    return fabs(x[0] * x[1] * x[2]) * I;
}

typedef struct {
    double om, mu0, D1, lext[3];
} ell_par;

/* mu(a) of the modified-gravity option at a^-3 = a3 */
static double ell_mu(double om, double mu0, double a3)
{
    return 1.0 + mu0 / (om * a3 + 1.0 - om);
}

/* state y = (x1, x2, x3, x1', x2', x3', D, D') in s = ln a */
static void ell_rhs(const ell_par *P, double s, const double y[8], double dy[8])
{
    double a3 = exp(-3.0 * s);
    double oma = P->om * a3 / (P->om * a3 + 1.0 - P->om);
    double damp = 2.0 - 1.5 * oma;
    double mu = ell_mu(P->om, P->mu0, a3);
    double x[3] = {y[0], y[1], y[2]};
    double delta = 1.0 / (x[0] * x[1] * x[2]) - 1.0;
    double dn = y[6] / P->D1;
    for (int i = 0; i < 3; ++i) {
        double al = orc_ell_alpha(x, i);
        dy[i] = y[3 + i];
        /* uniform excess delta/3 plus internal tide (alpha - 2/3) delta/2,
         * written as their sum alpha delta/2 */
        dy[3 + i] = -damp * y[3 + i] - 1.5 * oma * mu * x[i] * (0.5 * al * delta + dn * P->lext[i]);
    }
    dy[6] = y[7];
    dy[7] = -damp * y[7] + 1.5 * oma * mu * y[6];
}

static void ell_rk4(const ell_par *P, double s, double h, const double y[8], double out[8])
{
    double k1[8], k2[8], k3[8], k4[8], t[8];
    ell_rhs(P, s, y, k1);
    for (int c = 0; c < 8; ++c) t[c] = y[c] + 0.5 * h * k1[c];
    ell_rhs(P, s + 0.5 * h, t, k2);
    for (int c = 0; c < 8; ++c) t[c] = y[c] + 0.5 * h * k2[c];
    ell_rhs(P, s + 0.5 * h, t, k3);
    for (int c = 0; c < 8; ++c) t[c] = y[c] + h * k3[c];
    ell_rhs(P, s + h, t, k4);
    for (int c = 0; c < 8; ++c)
        out[c] = y[c] + h / 6.0 * (k1[c] + 2.0 * (k2[c] + k3[c]) + k4[c]);
}

/* D(a = 1) of the growing mode started as D = a at a_i, RK4 in s with the
 * same step as the ellipsoid (the normalisation both use) */
double orc_ell_growth1(double om, double mu0, double a_i, double h)
{
    double s = log(a_i);
    int n = (int)ceil(-s / h);
    double hh = -s / n;
    double y[2] = {a_i, a_i};
    for (int m = 0; m < n; ++m) {
        double ss = s + m * hh;
        double k[4][2], t[2];
        double oma, damp;
#define GROW(sv, yv, kv)                                                   \
        oma = om * exp(-3.0 * (sv)) / (om * exp(-3.0 * (sv)) + 1.0 - om); \
        damp = 2.0 - 1.5 * oma;                                            \
        kv[0] = yv[1];                                                     \
        kv[1] = -damp * yv[1] + 1.5 * oma * ell_mu(om, mu0, exp(-3.0 * (sv))) * yv[0];
        GROW(ss, y, k[0]);
        t[0] = y[0] + 0.5 * hh * k[0][0]; t[1] = y[1] + 0.5 * hh * k[0][1];
        GROW(ss + 0.5 * hh, t, k[1]);
        t[0] = y[0] + 0.5 * hh * k[1][0]; t[1] = y[1] + 0.5 * hh * k[1][1];
        GROW(ss + 0.5 * hh, t, k[2]);
        t[0] = y[0] + hh * k[2][0]; t[1] = y[1] + hh * k[2][1];
        GROW(ss + hh, t, k[3]);
#undef GROW
        for (int c = 0; c < 2; ++c)
            y[c] += hh / 6.0 * (k[0][c] + 2.0 * (k[1][c] + k[2][c]) + k[3][c]);
    }
    return y[0];
}

/* F = 1/D_c of the ellipsoid with eigenvalues lam (any order: the axis that
 * reaches zero first collapses), 0 without collapse by a_stop.  h: the RK4
 * step in ln a, shortened near collapse to kappa sqrt(x / |x''|) of the
 * smallest axis (the time over which its acceleration changes it: this
 * follows a regular crossing, where x'' stays finite, and the free-fall
 * approach of a nearly spherical collapse, where x ~ (s_c - s)^(2/3)).  A
 * step that ends with an axis <= 0 is bisected in length down to adjacent
 * doubles; an axis whose remaining time x / |x'| falls below 1e-12 (in ln a)
 * is taken as collapsed there.  *a_c receives the collapse scale factor (or
 * a_stop). */
double orc_ellipsoid_F(const double lam[3], double om, double mu0, double a_i, double a_stop, double h,
                       double kappa, double *a_c)
{
    ell_par P;
    P.om = om;
    P.mu0 = mu0;
    P.D1 = orc_ell_growth1(om, mu0, a_i, h);
    double dl = lam[0] + lam[1] + lam[2];
    for (int i = 0; i < 3; ++i)
        P.lext[i] = lam[i] - dl / 3.0;
    double y[8], yn[8], dy[8];
    for (int i = 0; i < 3; ++i) {
        y[i] = 1.0 - lam[i] * a_i / P.D1;
        y[3 + i] = -lam[i] * a_i / P.D1;
    }
    y[6] = a_i;
    y[7] = a_i;
    double s = log(a_i), se = log(a_stop);
    for (long step = 0; step < 100000000L && s < se; ++step) {
        int im = 0;
        for (int i = 1; i < 3; ++i)
            if (y[i] < y[im])
                im = i;
        if (y[im] < 1e-12 * fabs(y[3 + im]) && y[3 + im] < 0.0) {
            if (a_c)
                *a_c = exp(s);
            return P.D1 / y[6];
        }
        ell_rhs(&P, s, y, dy);
        double hs = h;
        double acc = fabs(dy[3 + im]);
        if (acc > 0.0) {
            double lim = kappa * sqrt(y[im] / acc);
            if (lim < hs)
                hs = lim;
        }
        if (s + hs > se)
            hs = se - s;
        ell_rk4(&P, s, hs, y, yn);
        double xmin = yn[0] < yn[1] ? yn[0] : yn[1];
        if (yn[2] < xmin) xmin = yn[2];
        if (!(xmin > 0.0)) {
            double lo = 0.0, hi = hs;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (!(mid > lo && mid < hi))
                    break;
                ell_rk4(&P, s, mid, y, yn);
                double xm = yn[0] < yn[1] ? yn[0] : yn[1];
                if (yn[2] < xm) xm = yn[2];
                if (xm > 0.0)
                    lo = mid;
                else
                    hi = mid;
            }
            ell_rk4(&P, s, hi, y, yn);
            if (a_c)
                *a_c = exp(s + hi);
            return P.D1 / yn[6];
        }
        s += hs;
        for (int c = 0; c < 8; ++c)
            y[c] = yn[c];
    }
    if (a_c)
        *a_c = a_stop;
    return 0.0;
}

/* The axes x_i = R_i/a of the ellipsoid at scale factor a_out (no collapse
 * check; for early-time checks).  Same integration as orc_ellipsoid_F. */
void orc_ellipsoid_axes(const double lam[3], double om, double mu0, double a_i, double a_out, double h,
                        double x_out[3], double *D_out)
{
    ell_par P;
    P.om = om;
    P.mu0 = mu0;
    P.D1 = orc_ell_growth1(om, mu0, a_i, h);
    double dl = lam[0] + lam[1] + lam[2];
    for (int i = 0; i < 3; ++i)
        P.lext[i] = lam[i] - dl / 3.0;
    double y[8], yn[8];
    for (int i = 0; i < 3; ++i) {
        y[i] = 1.0 - lam[i] * a_i / P.D1;
        y[3 + i] = -lam[i] * a_i / P.D1;
    }
    y[6] = a_i;
    y[7] = a_i;
    double s = log(a_i), se = log(a_out);
    int n = (int)ceil((se - s) / h);
    double hh = (se - s) / n;
    for (int m = 0; m < n; ++m) {
        ell_rk4(&P, s + m * hh, hh, y, yn);
        for (int c = 0; c < 8; ++c)
            y[c] = yn[c];
    }
    for (int i = 0; i < 3; ++i)
        x_out[i] = y[i];
    if (D_out)
        *D_out = y[6] / P.D1;
}

/* The ellipsoid table at nodes (delta, x, y) -> eigenvalues
 * l1 = (d + 2x + y)/3, l2 = (d - x + y)/3, l3 = (d - x - 2y)/3:
 * F[(ix * ny + iy) * nd + id] over the knots xk, yk, dk (already scaled). */
void orc_ellipsoid_table(int nx, int ny, int nd, const double *xk, const double *yk, const double *dk, double om,
                         double mu0, double a_i, double a_stop, double h, double kappa, double *F)
{
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int ix = 0; ix < nx; ++ix)
        for (int iy = 0; iy < ny; ++iy)
            for (int id = 0; id < nd; ++id) {
                double x = xk[ix], yv = yk[iy], d = dk[id];
                double lam[3] = {(d + 2.0 * x + yv) / 3.0, (d - x + yv) / 3.0, (d - x - 2.0 * yv) / 3.0};
                F[((size_t)ix * ny + iy) * nd + id] = orc_ellipsoid_F(lam, om, mu0, a_i, a_stop, h, kappa, NULL);
            }
}
