/*
 * pino_batch.h -- many realisations, each with all of its smoothing radii
 * resident in device memory, evaluated by one persistent kernel launch (an
 * addition to the paper's per-radius kernel, Sec. 4.1).
 *
 * A realisation carries its own cosmology (growth table of the context) and
 * particle count.  The plan cuts every realisation into tiles of particles;
 * the persistent kernel walks the static tile list (block b takes tiles b,
 * b + grid, ...) and, for each particle of a tile, applies all of the
 * realisation's radii in order with the running maximum held in registers,
 * writing Fmax, Rmax (and a_coll) once.  Results are identical to applying
 * the radii one by one with pino_collapse_eval (same device arithmetic, same
 * strict '>' order).
 *
 * Precision: PINO_FP64 contexts (double Hessians) and PINO_MIXED contexts
 * (float Hessians), Classic method.
 */
#ifndef PINO_BATCH_H
#define PINO_BATCH_H

#include <stdint.h>

#include "pino_collapse.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n;                  /* particles, >= 0 */
    int32_t n_radii;            /* >= 1 */
    const void *const *h;       /* host array of n_radii * 6 device pointers, radius-major:
                                   h[6*r + c] is component c (xx,yy,zz,xy,xz,yz) at radius r */
    int32_t cosmo;              /* growth table index of the context */
    int32_t radius_offset;      /* Rmax value of radius 0 (radius r writes radius_offset + r) */
    double *Fmax;               /* device in/out, n */
    int32_t *Rmax;              /* device in/out, n */
    double *a_coll;             /* device out, n; may be NULL */
} pino_realisation;

typedef struct pino_batch pino_batch;

/* Tile-size / grid choice.  tile = particles per tile (multiple of 256, 0 =
 * choose), blocks_per_cu (0 = choose).  With autotune != 0 the plan times
 * the candidates on the real data (the outputs are then overwritten, as by
 * any run) and keeps the fastest. */
typedef struct {
    int64_t tile;
    int32_t blocks_per_cu;
    int32_t autotune;
} pino_batch_tuning;

/* Build the static tile list and device descriptors (allocates; the only
 * call here that does).  flags: PINO_EVAL_RESET starts every particle from
 * Fmax = 0, Rmax = -1 (otherwise from the values in Fmax/Rmax);
 * PINO_EVAL_FINALIZE writes a_coll (required then) from the final maximum.
 * The realisation array and its pointer arrays are copied. */
pino_status pino_collapse_batch_plan(pino_ctx *ctx, const pino_realisation *reals, int32_t n_reals,
                                     uint32_t flags, const pino_batch_tuning *tuning, pino_batch **out);

/* One persistent launch on hip_stream.  Allocates nothing and issues no
 * memset, so it may be captured into a HIP graph. */
pino_status pino_collapse_batch_run(pino_batch *plan, void *hip_stream);

/* Capture pino_collapse_batch_run once into a HIP graph (first call) and
 * launch the graph on hip_stream. */
pino_status pino_collapse_batch_graph_launch(pino_batch *plan, void *hip_stream);

/* The configuration in use: tile, blocks per CU, grid, number of tiles. */
pino_status pino_collapse_batch_config(const pino_batch *plan, int64_t *tile, int32_t *blocks_per_cu,
                                       int32_t *grid, int64_t *n_tiles);

pino_status pino_collapse_batch_free(pino_batch *plan);

#ifdef __cplusplus
}
#endif

#endif /* PINO_BATCH_H */
