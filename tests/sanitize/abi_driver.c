/* Drives the argument validation of the collapse library's C ABI under the
 * host address and undefined-behaviour sanitizers (built by
 * tests/test_sanitizers.py).  Every call here is rejected by the pure host
 * checks before any HIP call, so it runs without a GPU.  Prints "ok". */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../include/pino_collapse.h"
#include "../../include/pino_interp.h"

static int expect(pino_status got, pino_status want, const char *what)
{
    if (got != want) {
        printf("%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, pino_collapse_last_error(NULL));
        return 1;
    }
    return 0;
}

int main(void)
{
    int bad = 0;
    pino_ctx *ctx = NULL;
    double a[8], D[8], Dbad[8];
    for (int k = 0; k < 8; ++k) {
        a[k] = 0.1 * (k + 1);
        D[k] = 0.1 * (k + 1);
        Dbad[k] = 0.1 * (8 - k);
    }
    pino_growth g = {8, a, D, 0.3};
    pino_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.abi_version = PINO_ABI_VERSION;
    cfg.n_cosmo = 1;
    cfg.growth = &g;
    bad |= expect(pino_collapse_init(NULL, &ctx), PINO_ERR_ARG, "NULL config");
    bad |= expect(pino_collapse_init(&cfg, NULL), PINO_ERR_ARG, "NULL out");
    cfg.abi_version = 99;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "version");
    cfg.abi_version = PINO_ABI_VERSION;
    cfg.method = 7;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "method");
    cfg.method = PINO_CLASSIC;
    cfg.precision = 9;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "precision");
    cfg.precision = PINO_FP64;
    g.D = Dbad;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "non-increasing D");
    g.D = D;
    g.n = 3;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "n < 4");
    g.n = 8;
    g.omega_m = NAN;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "omega_m NaN");
    g.omega_m = 1.5;
    cfg.method = PINO_CLASSIC_LCDM;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "LCDM omega_m > 1");
    g.omega_m = 0.3;
    cfg.method = PINO_TABULATED;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "tabulated without knots");
    double x[2] = {0, 1}, dl[4] = {0, 1, 2, 1.5};
    pino_table_knots tk = {2, 2, 4, x, x, dl};
    cfg.table = &tk;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "non-increasing delta knots");
    cfg.method = PINO_CLASSIC;
    cfg.table = NULL;
    cfg.precision = PINO_SURROGATE;
    unsigned char junk[16] = {0};
    cfg.mlp = junk;
    cfg.mlp_bytes = sizeof(junk);
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "surrogate blob");
    cfg.certify_rtol = -1.0;
    bad |= expect(pino_collapse_init(&cfg, &ctx), PINO_ERR_ARG, "certify_rtol");
    bad |= expect(pino_collapse_eval(NULL, NULL, 0, 0, NULL), PINO_ERR_ARG, "eval NULL ctx");
    bad |= expect(pino_collapse_free(NULL), PINO_OK, "free NULL");
    if (!pino_collapse_last_error(NULL))
        bad = 1;
    /* stand-alone interpolators: bad sizes and NULL pointers */
    bad |= expect(pino_spline_build(0, NULL, NULL, 8, NULL, NULL, NULL), PINO_ERR_ARG, "spline_build NULL");
    bad |= expect(pino_table_eval(0, x, 1, x, 2, dl, 4, NULL, NULL, NULL, NULL, NULL, 0, NULL), PINO_ERR_ARG,
                  "table_eval nx 1");
    bad |= expect(pino_table_interp_noalloc(0, x, 2, x, 2, dl, 4, NULL, NULL, NULL, NULL, NULL, 4, NULL),
                  PINO_ERR_ARG, "noalloc NULL F");
    if (bad)
        return 1;
    printf("ok\n");
    return 0;
}
