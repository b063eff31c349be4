/*
 * pino_field.h -- the Hessians of the smoothed potential built on the device
 * from the linear density field, and the collapse of a list of radii fed
 * from them without leaving the device.  Sec. 3 of the paper builds the six
 * second derivatives per radius with FFTs; the offloaded collapse stage then
 * moves them between host and device, the cost its conclusions name as the
 * next thing to remove.
 *
 * Field: delta(k), the real-FFT half grid of the linear density contrast on
 * a periodic n^3 grid of side L, complex128 [n][n][n/2+1] (x slowest, z
 * halved; forward transform unnormalised, the layout numpy.fft.rfftn and
 * torch.fft.rfftn return).  For smoothing radius R (Gaussian window):
 *
 *   H_ij(x) = (1/n^3) sum_k (k_i k_j / k^2) exp(-k^2 R^2 / 2) delta(k) e^{ik.x},
 *
 * with H_ij(k = 0) = 0, wavenumbers 2 pi/L times (0, 1, ..., n/2 - 1, -n/2,
 * ..., -1) along x and y and (0, ..., n/2) along z; so tr H = delta_R
 * (nabla^2 phi = delta).  For an even side, modes at the Nyquist index along
 * any axis are dropped (+n/2 and -n/2 alias there, so the derivative of such
 * a wave is not defined on the grid).  Output H: (6, n^3) SoA, components
 * xx, yy, zz, xy, xz, yz, particle (ix * n + iy) * n + iz, FP64 (or FP32 for
 * the single-precision variant), the layout pino_collapse_eval reads.
 */
#ifndef PINO_FIELD_H
#define PINO_FIELD_H

#include <stdint.h>

#include "pino_collapse.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pino_field pino_field;

/* Plans for an n^3 grid of side box (n in [2, 1024], box > 0) on a device:
 * allocates the k-space work buffer (6 n^2 (n/2+1) complex128) and a
 * Hessian buffer (6 n^3 doubles) and creates the batched complex-to-real FFT
 * plans (FP64 and FP32).  The only call here that allocates. */
pino_status pino_field_create(int32_t device, int32_t n_side, double box, pino_field **out);

/* H (device, 6 n^3 doubles, caller-owned) for radius R >= 0 from delta_k
 * (device, caller-owned, not modified), asynchronously on hip_stream
 * (NULL = the default stream). */
pino_status pino_field_hessian(pino_field *f, const void *delta_k, double R, double *H, void *hip_stream);

/* The same in FP32 arithmetic (k-space products and transform), H float. */
pino_status pino_field_hessian_f32(pino_field *f, const void *delta_k, double R, float *H, void *hip_stream);

/* For r = 0 .. n_radii - 1: the Hessian at radii[r] into the field's own
 * buffer (FP64 for a PINO_FP64 context, FP32 for PINO_MIXED and
 * PINO_SURROGATE), then pino_collapse_eval of items[r] with its h[] pointing
 * there.  items[r] supplies everything else of an eval item (n must be n^3;
 * cosmo, radius_index, sigma_R, table_F, Fmax, Rmax, a_coll), its h[] is
 * ignored.  flags: PINO_EVAL_RESET applies to the first radius,
 * PINO_EVAL_FINALIZE to the last, PINO_EVAL_SYNC waits at the end.
 * Allocates nothing. */
pino_status pino_field_collapse(pino_field *f, pino_ctx *ctx, const void *delta_k, const double *radii,
                                const pino_item *items, int32_t n_radii, uint32_t flags, void *hip_stream);

/* NULL-safe; the message of the last failed call on f (or of the last failed
 * create when f is NULL). */
pino_status pino_field_free(pino_field *f);
const char *pino_field_last_error(const pino_field *f);

#ifdef __cplusplus
}
#endif

#endif /* PINO_FIELD_H */
