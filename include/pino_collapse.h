/*
 * pino_collapse.h -- C ABI of the MI355X collapse-time library.
 *
 * For every particle and every smoothing radius the library takes the six
 * components of the Hessian of the smoothed linear potential, finds its
 * eigenvalues, computes the growth factor at collapse, converts it to a
 * collapse scale factor through the inverse of the linear growth table, and
 * keeps the earliest collapse over the radii processed so far (Sec. 3 and
 * Sec. 4.1 of Lepinzan et al., "Accelerating cosmological simulations on
 * GPUs: a portable approach using OpenMP").
 *
 *   Classic   : third-order LPT collapse condition of the homogeneous
 *               ellipsoid, solved for its smallest positive root (Sec. 3).
 *   Tabulated : collapse function tabulated over delta = l1 + l2 + l3,
 *               x = l1 - l2, y = l2 - l3 (eigenvalues in descending order),
 *               interpolated with a natural cubic spline in delta and
 *               bilinearly in (x, y); the delta splines are rebuilt on the
 *               device for every radius (Sec. 3, Sec. 4.2).
 *
 * Quantities (per particle i):
 *   F      = 1 / D_c, the inverse growth factor at collapse ("inverse
 *            collapse time"); 0 when the particle never collapses.
 *   Fmax   = max over the radii applied so far of F (strict '>' update, so
 *            the first radius wins exact ties; NaN never updates).
 *   Rmax   = radius_index of the item that set Fmax, -1 if none.
 *   a_coll = a(D_c) of that radius through the natural cubic spline of the
 *            growth table (a_k as a function of D_k); +inf when D_c is past
 *            the last tabulated D (collapse after the end of the table);
 *            clamped to a_0 when D_c is below the first tabulated D.
 *            z_coll = 1 / a_coll - 1.
 *
 * Memory: every Hessian and output buffer is device memory owned by the
 * caller.  Hessians are structure-of-arrays, one contiguous array per
 * component (xx, yy, zz, xy, xz, yz), element i of each belonging to
 * particle i.  Host arrays handed to pino_collapse_init are copied before it
 * returns.  The library owns only what init allocates.
 *
 * Errors: every call returns a pino_status; no exception or abort crosses the
 * ABI.  pino_collapse_last_error() returns a message for the last failure.
 * After PINO_ERR_HIP the context answers PINO_ERR_STATE until it is freed.
 *
 * Threads: a context may be used by one host thread at a time.
 */
#ifndef PINO_COLLAPSE_H
#define PINO_COLLAPSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PINO_ABI_VERSION 1

typedef enum {
    PINO_OK = 0,
    PINO_ERR_ARG = 1,          /* invalid argument; nothing was enqueued */
    PINO_ERR_ALLOC = 2,        /* device or host allocation failed */
    PINO_ERR_HIP = 3,          /* a HIP call failed; context is now unusable */
    PINO_ERR_STATE = 4,        /* context unusable after an earlier HIP error */
    PINO_ERR_UNSUPPORTED = 5   /* combination of options not implemented */
} pino_status;

typedef enum { PINO_CLASSIC = 0, PINO_TABULATED = 1 } pino_method;

/* Arithmetic of the evaluation.
 *   PINO_FP64      : FP64 Hessians, FP64 throughout.
 *   PINO_MIXED     : FP32 Hessians.  Classic: eigenvalues and interpolation
 *                    in FP32, FP64 for nearly degenerate eigenvalues and for
 *                    the final polish of the collapse root.  Tabulated: the
 *                    Hessians widened to FP64 for the eigenvalues and the
 *                    cell search, the table read from an FP32 copy built on
 *                    the device each radius (F and the spline second
 *                    derivatives rounded to FP32), the interpolation in FP64.
 *                    a(D) in FP32 for both.
 *   PINO_SURROGATE : FP32 Hessians; a small network predicts the collapse
 *                    growth factor and one FP64 Newton step refines it; the
 *                    result is accepted only if the first root of the
 *                    collapse condition provably lies within certify_rtol of
 *                    it.  Particles that fail are queued and take the full
 *                    FP64 solve in a second kernel of the same eval (items
 *                    are processed in chunks of 2^24 particles, the queue's
 *                    size).  Classic only; weights from pino_mlp.h. */
typedef enum { PINO_FP64 = 0, PINO_MIXED = 1, PINO_SURROGATE = 2 } pino_precision;

/* eval flags */
#define PINO_EVAL_RESET 1u     /* set Fmax = 0, Rmax = -1, a_coll = +inf before applying the item */
#define PINO_EVAL_SYNC 2u      /* wait for the stream before returning */
#define PINO_EVAL_FINALIZE 4u  /* after applying the item, set a_coll (non-NULL) for every particle
                                  from the running maximum: a(1/Fmax), or +inf where Fmax == 0.
                                  Because a(D) is increasing, this equals what per-update a_coll
                                  gives, bit for bit; callers may pass a_coll = NULL for all but
                                  the last radius and FINALIZE on the last one. */

/* One linear growth table: n >= 4 knots, a and D strictly increasing and
 * finite (host pointers, copied by init).  The library builds the natural
 * spline a(D) from it on the device.  omega_m is the matter density of the
 * cosmology (an input of the surrogate network; otherwise unused). */
typedef struct {
    int32_t n;
    const double *a;
    const double *D;
    double omega_m;
} pino_growth;

/* Knots of the collapse table in units of sigma(R): each item's sigma_R
 * multiplies them.  nx, ny >= 2 and nd >= 4 strictly increasing finite host
 * values, copied by init; nx * ny * nd <= 2^24. */
typedef struct {
    int32_t nx, ny, nd;
    const double *x, *y, *delta;
} pino_table_knots;

typedef struct {
    int32_t abi_version;             /* PINO_ABI_VERSION */
    int32_t method;                  /* pino_method */
    int32_t precision;               /* pino_precision */
    int32_t device;                  /* HIP device ordinal */
    int32_t n_cosmo;                 /* >= 1 growth tables, one per cosmology */
    const pino_growth *growth;       /* host array of n_cosmo tables, each n <= 2048 */
    const pino_table_knots *table;   /* PINO_TABULATED only, else NULL */
    const void *mlp;                 /* PINO_SURROGATE only: blob from pino_mlp_export */
    int64_t mlp_bytes;
    double certify_rtol;             /* PINO_SURROGATE: certified relative accuracy
                                        of the collapse growth factor (the root is
                                        bracketed within u (1 -/+ rtol)); <= 0
                                        selects 5e-7 */
} pino_config;

/* One realisation at one smoothing radius. */
typedef struct {
    int64_t n;                       /* particles, >= 0 */
    const void *h[6];                /* device: double (PINO_FP64) or float
                                        (PINO_MIXED, PINO_SURROGATE), each n long */
    int32_t cosmo;                   /* growth table index, 0 <= cosmo < n_cosmo */
    int32_t radius_index;            /* written to Rmax on update, >= 0 */
    double sigma_R;                  /* rms of the smoothed field at this radius
                                        (> 0; scales table knots and network inputs) */
    const double *table_F;           /* PINO_TABULATED: device, F at the knots
                                        scaled by sigma_R, [nx][ny][nd] row-major */
    double *Fmax;                    /* device in/out, n */
    int32_t *Rmax;                   /* device in/out, n */
    double *a_coll;                  /* device in/out, n; may be NULL */
} pino_item;

typedef struct pino_ctx pino_ctx;

/* Create a context on cfg->device: copy the growth tables (and table knots
 * or network weights) to the device and build their splines there.  Waits for
 * that work to finish.  On failure *out is NULL and the status says why. */
pino_status pino_collapse_init(const pino_config *cfg, pino_ctx **out);

/* Apply n_items items, in order, on hip_stream (a hipStream_t; NULL means the
 * device's null stream).  Asynchronous unless PINO_EVAL_SYNC.  Items may mix
 * realisations and cosmologies; items whose outputs overlap are applied in
 * the order given.  Allocates nothing. */
pino_status pino_collapse_eval(pino_ctx *ctx, const pino_item *items, int32_t n_items, uint32_t flags,
                               void *hip_stream);

/* Release everything init allocated.  NULL-safe.  Waits for the context's
 * outstanding work on the device. */
pino_status pino_collapse_free(pino_ctx *ctx);

/* Message for the last failure on ctx, or of the last failed init on this
 * thread when ctx is NULL.  Never NULL; valid until the next call. */
const char *pino_collapse_last_error(const pino_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PINO_COLLAPSE_H */
