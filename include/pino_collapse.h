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
 * Threads and streams: a context may be used by one host thread at a time.
 * Successive evals may use different streams.  A context that holds device
 * scratch of its own (the Tabulated method's per-radius table, the
 * surrogate's queue and counters) orders its evals across streams: an eval
 * on a stream other than the previous eval's waits for that eval's work.
 * While the caller captures a stream into a graph no such ordering is
 * inserted; the caller then orders the graph against other streams.
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

/* Collapse method.
 *   PINO_CLASSIC      : the third-order LPT condition with its Einstein-de
 *                       Sitter time coefficients (Sec. 3).
 *   PINO_TABULATED    : the (delta, x, y) table (Sec. 3, Sec. 4.2).
 *   PINO_CLASSIC_LCDM : the same LPT condition with the time coefficients
 *                       of flat LCDM: its second- and third-order terms are
 *                       scaled by the ratios of their LCDM growth functions
 *                       to the Einstein-de Sitter ones at the epoch of the
 *                       growth factor D (Sec. 3 names the LPT formulation;
 *                       the cosmology dependence is an addition).  The ratios
 *                       are integrated on the device at init for each growth
 *                       table's omega_m (0 < omega_m <= 1; flat, no
 *                       radiation) at its knots and interpolated in D.  FP64
 *                       or PINO_SURROGATE (not PINO_MIXED); per-radius evals
 *                       only (no batch plan). */
typedef enum { PINO_CLASSIC = 0, PINO_TABULATED = 1, PINO_CLASSIC_LCDM = 2 } pino_method;

/* Arithmetic of the evaluation.
 *   PINO_FP64      : FP64 Hessians, FP64 throughout.
 *   PINO_MIXED     : FP32 Hessians, eigenvalues and interpolation in FP32,
 *                    FP64 for nearly degenerate eigenvalues.  Classic: FP64
 *                    for the final polish of the collapse root.  Tabulated:
 *                    the cell search in FP32 copies of the scaled knots, the
 *                    table read from an FP32 copy built on the device each
 *                    radius (F and the spline second derivatives rounded to
 *                    FP32), spline and bilinear interpolation in FP32.
 *                    a(D) in FP32 for both.
 *   PINO_SURROGATE : FP64 Hessians and FP64 eigenvalues; a small network
 *                    (BF16 matrix-core inference) predicts the collapse
 *                    growth factor and one FP64 Newton step refines it; the
 *                    result is accepted only if the first root of the
 *                    particle's collapse condition provably lies within
 *                    certify_rtol of it.  Particles that fail are queued by
 *                    the workgroup that visited them, which then gives them
 *                    the full FP64 solve in the same launch (items are
 *                    processed in chunks of 2^24 particles, the queue's
 *                    size).  Classic or Classic-LCDM (the network then
 *                    predicts the LCDM condition's root; its omega_m input
 *                    matters); weights from pino_mlp.h. */
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
 * cosmology: an input of the surrogate network, and the cosmology of the
 * PINO_CLASSIC_LCDM time coefficients; otherwise unused. */
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
    const void *h[6];                /* device: double (PINO_FP64, PINO_SURROGATE)
                                        or float (PINO_MIXED), each n long */
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

/* Create a context on cfg->device (Sec. 3, Sec. 4.2).
 *
 * Copies the growth tables to the device and builds there, for each, the
 * natural cubic spline of a as a function of D that turns the growth factor
 * at collapse into a_coll (Sec. 3: the collapse time follows from a spline
 * of the linear growth table; Sec. 4.2: splines built and evaluated on the
 * device).  A Tabulated context also copies its table knots and allocates
 * the per-radius table the evals rebuild; a surrogate context converts the
 * network weights to its matrix-core fragments and allocates its queue.
 * Waits for that work to finish.
 *
 * cfg: host pointer, read during the call only (every host array it points
 * to is copied).  *out: the new context, owned by the caller until
 * pino_collapse_free.  Errors: PINO_ERR_ARG (invalid configuration, checked
 * before any HIP call), PINO_ERR_UNSUPPORTED (knots that do not fit the
 * kernels' LDS), PINO_ERR_HIP or PINO_ERR_ALLOC; on failure *out is NULL
 * and pino_collapse_last_error(NULL) says why. */
pino_status pino_collapse_init(const pino_config *cfg, pino_ctx **out);

/* Apply n_items items, in order, on hip_stream (Sec. 3, Sec. 4.1).
 *
 * Per particle of each item: the eigenvalues of its Hessian, sorted in
 * descending order (Sec. 3, an analytic method); the growth factor at
 * collapse from the Classic third-order LPT condition or from the Tabulated
 * spline/bilinear interpolation (Sec. 3, Sec. 4.2); F = 1/D_c; the strict
 * '>' update of the per-element maxima Fmax and Rmax, and a_coll (Sec. 4.1:
 * the kernel's read/modify/write of two output arrays per element).
 * Tabulated items first rebuild the natural splines of their table on the
 * device (Sec. 4.2).
 *
 * items: host array of n_items items, read during the call; their device
 * arrays stay owned by the caller and must stay valid until the stream has
 * run the work.  hip_stream: a hipStream_t, NULL for the device's null
 * stream.  Asynchronous unless PINO_EVAL_SYNC.  Items may mix realisations
 * and cosmologies; items whose outputs overlap are applied in the order
 * given.  Allocates nothing.  Errors: PINO_ERR_ARG (nothing enqueued),
 * PINO_ERR_STATE (context broken), PINO_ERR_HIP (launch failure; the context
 * is broken from then on). */
pino_status pino_collapse_eval(pino_ctx *ctx, const pino_item *items, int32_t n_items, uint32_t flags,
                               void *hip_stream);

/* Release everything init allocated (the device copies of the growth
 * tables, splines and table of Sec. 3 and Sec. 4.2).  NULL-safe.  Waits for
 * the context's device first.  Returns PINO_ERR_HIP if that wait reports an
 * error; the memory is released either way. */
pino_status pino_collapse_free(pino_ctx *ctx);

/* Fill a Tabulated table from the homogeneous-ellipsoid collapse (Sec. 3:
 * the table of the Tabulated method comes from integrating nine ODEs with
 * fourth-order Runge-Kutta until the density diverges).  For every node
 * (x_ix, y_iy, delta_id) of the context's table knots scaled by sigma_R, the
 * eigenvalues l1 = (delta + 2x + y)/3, l2 = (delta - x + y)/3,
 * l3 = (delta - x - 2y)/3 set the linear deformation of a unit sphere in the
 * flat LCDM cosmology of growth table `cosmo` (its omega_m, 0 < omega_m <= 1);
 * the axes, the scale factor and the linear growth are integrated from
 * a = 1e-7 with the ellipsoid's own gravity and the linear external tide
 * until the first axis reaches zero, and F = 1/D_c is written, D_c the linear
 * growth factor then (normalised to 1 today); 0 if no axis collapses by
 * a = 10.  table_F: device, caller-owned, nx * ny * nd doubles in the layout
 * pino_item.table_F takes.  One thread per node; asynchronous on hip_stream;
 * allocates nothing.  PINO_ERR_ARG for another method, a bad index or
 * omega_m, a non-positive sigma_R or NULL table_F. */
pino_status pino_collapse_ellipsoid_table(pino_ctx *ctx, int32_t cosmo, double sigma_R, double *table_F,
                                          void *hip_stream);

/* The same table under a modified-gravity option (the Tabulated method is
 * the one meant for modified gravity, Sec. 3, where the LPT condition does
 * not apply): the gravity of the density perturbations -- the ellipsoid's
 * excess and internal tide, the external tide and the linear growth that
 * normalises D -- is scaled by mu(a) = 1 + mu0 / E(a)^2, E^2 = omega_m a^-3
 * + 1 - omega_m (in flat LCDM, 1 + mu0 Omega_L(a)/Omega_L today: standard
 * gravity early, the departure growing as the cosmological constant takes
 * over); the background expansion is unchanged.  mu0 = 0 gives
 * pino_collapse_ellipsoid_table bit for bit.  PINO_ERR_ARG also when mu0 is
 * not finite, not above -(1 - omega_m) (mu must stay positive), or not 0
 * with omega_m = 1.  The growth table of the context that inverts D_c
 * should be the one of the same option.  The option's D(a = 1) is
 * integrated on the host at each call with mu0 != 0 (a few ms). */
pino_status pino_collapse_ellipsoid_table_mg(pino_ctx *ctx, int32_t cosmo, double sigma_R, double mu0,
                                             double *table_F, void *hip_stream);

/* The LCDM time coefficients of a PINO_CLASSIC_LCDM context at the knots of
 * growth table `cosmo`: k2, k3a, k3b (host arrays of that table's n
 * doubles, written) are the second-order, third-order determinant-type and
 * third-order mixed growth divided by their Einstein-de Sitter values
 * (-(3/7) D^2, -(1/3) D^3, (10/21) D^3).  Waits for the context's device.
 * PINO_ERR_ARG for another method, a bad index or NULL outputs. */
pino_status pino_collapse_lpt_coefficients(pino_ctx *ctx, int32_t cosmo, double *k2, double *k3a, double *k3b);

/* Message for the last failure on ctx, or of the last failed init on this
 * thread when ctx is NULL.  Never NULL; owned by the library and valid until
 * the next call on the same context (or thread).  Not a method of the paper:
 * the error channel of this ABI. */
const char *pino_collapse_last_error(const pino_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PINO_COLLAPSE_H */
