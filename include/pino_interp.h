/*
 * pino_interp.h -- the device interpolators of the collapse path as
 * stand-alone calls, for the interpolation benchmarks of Sec. 4.3 (a 1-D
 * cubic spline on 512 random knots, and the 64 x 64 table of 128-knot
 * splines with bilinear interpolation between rows), validated there against
 * GSL on analytic functions.
 *
 * Spline: natural cubic spline (second derivative 0 at both ends, the GSL
 * "cspline" the paper replaces) through (x[k], y[k]), k < n, x strictly
 * increasing.  A query q in [x_i, x_{i+1}) uses interval i; q at or beyond
 * the last knot uses the last interval and q below the first the first (the
 * end cubic is extended).
 *
 * Table: values F[(ix * ny + iy) * nd + id] at knots xk[ix], yk[iy], dk[id];
 * a query (x, y, d) evaluates the natural splines in d of the four rows at
 * the corners of the (x, y) cell and interpolates them bilinearly.  The cell
 * fractions are clamped to [0, 1] and d to [dk[0], dk[nd-1]]; the result is
 * clamped to >= 0 (the table of the Tabulated collapse holds F = 1/D_c >= 0).
 * This is the interpolator the Tabulated collapse kernel uses.
 *
 * All arrays are device memory owned by the caller; calls are asynchronous
 * on hip_stream (NULL = default stream) and allocate nothing.  Errors:
 * PINO_ERR_ARG for bad sizes or NULL pointers (checked before any HIP
 * call), PINO_ERR_HIP for launch failures; pino_interp_last_error() gives
 * the message (per host thread).
 */
#ifndef PINO_INTERP_H
#define PINO_INTERP_H

#include <stdint.h>

#include "pino_collapse.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Second derivatives M[n] of the natural spline; work: n doubles of scratch.
 * 2 <= n <= 2048 (the evaluator stages the knots in LDS). */
pino_status pino_spline_build(int32_t device, const double *x, const double *y, int32_t n, double *M, double *work,
                              void *hip_stream);

/* out[i] = spline(q[i]), i < m (knots staged in LDS). */
pino_status pino_spline_eval(int32_t device, const double *x, const double *y, const double *M, int32_t n,
                             const double *q, double *out, int64_t m, void *hip_stream);

/* The interleaved table the evaluator reads: tab[2 * ((ix * ny + iy) * nd +
 * id) + {0, 1}] = (F, M), M the natural-spline second derivatives of each
 * d-row; tab holds 2 nx ny nd doubles, work nx ny nd doubles of scratch.
 * 2 <= nx, ny <= 1024, 2 <= nd <= 4096. */
pino_status pino_table_build(int32_t device, int32_t nx, int32_t ny, int32_t nd, const double *dk, const double *F,
                             double *tab, double *work, void *hip_stream);

/* out[i] = table(qx[i], qy[i], qd[i]), i < m. */
pino_status pino_table_eval(int32_t device, const double *xk, int32_t nx, const double *yk, int32_t ny,
                            const double *dk, int32_t nd, const double *tab, const double *qx, const double *qy,
                            const double *qd, double *out, int64_t m, void *hip_stream);

/* pino_table_build followed by pino_table_eval in one call that allocates
 * nothing and needs no work or table buffer from the caller: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The spline coefficients
 * and the interleaved (F, M) table are built in a static device array of
 * the library (about 16.1 MiB per GPU, held until the process ends): at
 * most 2^20 table values (nx * ny * nd) and nd <= 4096, PINO_ERR_ARG beyond.
 * F: the table values F[(ix * ny + iy) * nd + id] (device, caller-owned);
 * knots, queries and out as for pino_table_eval.  Every call on a GPU uses
 * that GPU's one array, whose contents the call rewrites before reading, so
 * calls that overlap on one GPU (other threads, or streams not ordered with
 * each other) race and must not be made. */
pino_status pino_table_interp_noalloc(int32_t device, const double *xk, int32_t nx, const double *yk, int32_t ny,
                                      const double *dk, int32_t nd, const double *F, const double *qx,
                                      const double *qy, const double *qd, double *out, int64_t m,
                                      void *hip_stream);

const char *pino_interp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PINO_INTERP_H */
