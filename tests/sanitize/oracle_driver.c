/* Drives the oracle's C functions under the host address and
 * undefined-behaviour sanitizers (built by tests/test_sanitizers.py with
 * gcc).  Covers the degenerate and ragged inputs the oracle is used on:
 * 2-knot splines, repeated and zero eigenvalues, NaN Hessians, empty and
 * one-element radius updates, the LCDM coefficients and the ellipsoid
 * integration (coarse step).  Prints "ok" and returns 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_eig3(const double h[6], double lam[3]);
double orc_collapse_D(const double lam[3], int *found);
int orc_spline_natural(int n, const double *x, const double *y, double *M);
double orc_spline_eval(int n, const double *x, const double *y, const double *M, double q);
double orc_growth_invert(int nk, const double *D, const double *a, const double *M, double Dc);
int orc_table_build(int nx, int ny, int nd, const double *dk, const double *F, double *M);
double orc_table_F(int nx, int ny, int nd, const double *xk, const double *yk, const double *dk, const double *F,
                   const double *M, const double lam[3]);
void orc_update_radius(int64_t n, const double *hxx, const double *hyy, const double *hzz, const double *hxy,
                       const double *hxz, const double *hyz, int32_t radius_index, int method, int nk,
                       const double *gD, const double *ga, const double *gM, int nx, int ny, int nd,
                       const double *xk, const double *yk, const double *dk, const double *tF, const double *tM,
                       int reset, double *Fmax, int32_t *Rmax, double *acoll);
int orc_lpt_growth(double om, int nk, const double *ak, double *k2, double *k3a, double *k3b);
double orc_collapse_D_lcdm(const double lam[3], int nk, const double *D, const double *k2, const double *m2,
                           const double *k3a, const double *m3a, const double *k3b, const double *m3b, int *found);
double orc_ellipsoid_F(const double lam[3], double om, double mu0, double a_i, double a_stop, double h, double kappa,
                       double *a_c);
double orc_growth_D(double om, double a);

int main(void)
{
    const double hs[][6] = {{1, 1, 1, 0, 0, 0}, {0, 0, 0, 0, 0, 0}, {2, -1, 0.5, 0.3, -0.2, 0.1},
                            {NAN, 0, 0, 0, 0, 0}, {1e-300, 0, 0, 0, 0, 0}, {3, 3, -1, 0, 0, 0}};
    int nh = (int)(sizeof(hs) / sizeof(hs[0]));
    for (int k = 0; k < nh; ++k) {
        double lam[3];
        int found;
        orc_eig3(hs[k], lam);
        (void)orc_collapse_D(lam, &found);
    }
    /* splines: 2 knots, and a growth table */
    double x2[2] = {0.0, 1.0}, y2[2] = {1.0, 2.0}, m2[2];
    if (orc_spline_natural(2, x2, y2, m2) != 0)
        return 1;
    (void)orc_spline_eval(2, x2, y2, m2, 5.0);
    enum { NK = 64 };
    double a[NK], D[NK], M[NK];
    for (int k = 0; k < NK; ++k) {
        a[k] = exp(log(1e-3) + k * (-log(1e-3)) / (NK - 1));
        D[k] = orc_growth_D(0.3, a[k]);
    }
    if (orc_spline_natural(NK, D, a, M) != 0)
        return 2;
    (void)orc_growth_invert(NK, D, a, M, 2.0);
    (void)orc_growth_invert(NK, D, a, M, 1e-9);
    /* a 2 x 2 x 4 table */
    double xk[2] = {0, 1}, yk[2] = {0, 1}, dk[4] = {-1, 0, 1, 2}, F[16], TM[16];
    for (int i = 0; i < 16; ++i)
        F[i] = 0.1 * i;
    if (orc_table_build(2, 2, 4, dk, F, TM) != 0)
        return 3;
    for (int k = 0; k < nh; ++k) {
        double lam[3];
        orc_eig3(hs[k], lam);
        (void)orc_table_F(2, 2, 4, xk, yk, dk, F, TM, lam);
    }
    /* radius updates: n = 0, 1 and a few, both methods */
    for (int method = 0; method < 2; ++method)
        for (int n = 0; n <= 5; n += 5) {
            double *h = malloc(sizeof(double) * 6 * (n + 1));
            double *Fm = malloc(sizeof(double) * (n + 1)), *ac = malloc(sizeof(double) * (n + 1));
            int32_t *Rm = malloc(sizeof(int32_t) * (n + 1));
            for (int i = 0; i < 6 * (n + 1); ++i)
                h[i] = (i % 7) * 0.3 - 0.5;
            orc_update_radius(n, h, h + n, h + 2 * n, h + 3 * n, h + 4 * n, h + 5 * n, 0, method, NK, D, a, M, 2, 2,
                              4, xk, yk, dk, F, TM, 1, Fm, Rm, ac);
            free(h);
            free(Fm);
            free(ac);
            free(Rm);
        }
    /* LCDM coefficients and root */
    double k2[NK], k3a[NK], k3b[NK], s2[NK], s3a[NK], s3b[NK];
    if (orc_lpt_growth(0.3, NK, a, k2, k3a, k3b) != 0)
        return 4;
    orc_spline_natural(NK, D, k2, s2);
    orc_spline_natural(NK, D, k3a, s3a);
    orc_spline_natural(NK, D, k3b, s3b);
    {
        double lam[3] = {1.0, 0.5, -0.2};
        int found;
        (void)orc_collapse_D_lcdm(lam, NK, D, k2, s2, k3a, s3a, k3b, s3b, &found);
    }
    /* ellipsoid: a sphere and an ellipsoid with a coarse step */
    {
        double sph[3] = {1, 1, 1}, ell[3] = {1.0, 0.5, -0.2}, ac;
        (void)orc_ellipsoid_F(sph, 1.0, 0.0, 1e-4, 10.0, 5e-2, 0.1, &ac);
        (void)orc_ellipsoid_F(ell, 0.3, 0.0, 1e-4, 10.0, 5e-2, 0.1, &ac);
        (void)orc_ellipsoid_F(ell, 0.3, 0.4, 1e-4, 10.0, 5e-2, 0.1, &ac);
    }
    printf("ok\n");
    return 0;
}
