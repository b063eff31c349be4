/*
 * pino_mlp.h -- the learned surrogate of the Classic collapse (an addition:
 * the paper does not use one).
 *
 * Network: 4 -> 64 -> 64 -> 64 -> 1, ReLU hidden activations.
 *   input  x = (l1/sigma_R, l2/sigma_R, l3/sigma_R, (Omega_m - 0.3)/0.05),
 *          eigenvalues of the Hessian in descending order (Sec. 3);
 *   output y ~ w = 1/(l1 D_c), so the predicted growth factor at collapse is
 *          D^ = 1/(l1 y) (w is scale free: the LPT collapse condition is
 *          homogeneous of degree -1 in the eigenvalues).
 * Parameters, FP32, 8705 values in this order: W1[64][4], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4 (W[out][in]).
 *
 * The network is only consulted where it can help: l1 <= 0 never collapses
 * (F = 0 exactly) and l1 < 0.1 max|l| takes the full solve directly.
 * Everything here runs on the device; host pointers are marked.
 */
#ifndef PINO_MLP_H
#define PINO_MLP_H

#include <stdint.h>

#include "pino_collapse.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PINO_MLP_PARAMS 8705

typedef struct pino_mlp pino_mlp;

/* FP32 master parameters (He-uniform from seed, zero biases, b4 = 1) and Adam
 * state on `device`. */
pino_status pino_mlp_create(int32_t device, uint64_t seed, pino_mlp **out);

/* Copy parameters in / out (host arrays of PINO_MLP_PARAMS floats). */
pino_status pino_mlp_set_params(pino_mlp *m, const float *host_params);
pino_status pino_mlp_get_params(pino_mlp *m, float *host_params);

/* FP32 forward: x device [n][4], y device [n]. */
pino_status pino_mlp_forward(pino_mlp *m, const float *x, float *y, int64_t n, void *hip_stream);

/* Mean relative squared error L = (1/n) sum ((y_i - w_i)/w_i)^2 over samples
 * with w_i > 0 (others ignored, n counts all), its gradient with respect to
 * the parameters (device, PINO_MLP_PARAMS floats, overwritten) and L (device,
 * one float).  Deterministic: per-block partial sums reduced in fixed order.
 * 0 < n <= 65536. */
pino_status pino_mlp_grad(pino_mlp *m, const float *x, const float *w, int64_t n, float *grad, float *loss,
                          void *hip_stream);

/* BF16 forward for training (on = 1; off = 0, the default): pino_mlp_grad
 * then evaluates the network under the BF16 rounding rule of the surrogate:
 * the weights of the two 64 x 64 layers, and the inputs of those layers and
 * of the output layer (the ReLU outputs of layers 1, 2 and 3), rounded to
 * BF16 (nearest even, ties to even); FP32 accumulation; layer 1's weights
 * and inputs, the output layer's weights and every bias kept FP32.  The
 * backward pass treats the rounding as the identity (straight-through) and
 * updates the FP32 master parameters.  PINO_ERR_ARG for other values of on. */
pino_status pino_mlp_set_bf16_forward(pino_mlp *m, int32_t on);

/* One Adam step (bias-corrected; step counter kept in the handle) with the
 * given gradient (device). */
pino_status pino_mlp_adam(pino_mlp *m, const float *grad, float lr, float beta1, float beta2, float eps,
                          void *hip_stream);

/* grad + adam on one minibatch; loss (device, may be NULL). */
pino_status pino_mlp_train_step(pino_mlp *m, const float *x, const float *w, int64_t n, float lr, float *loss,
                                void *hip_stream);

/* Serialize the current parameters into a blob for pino_config.mlp (host
 * memory).  *needed receives the size; blob may be NULL to query it. */
pino_status pino_mlp_export(pino_mlp *m, void *blob, int64_t bytes, int64_t *needed);

pino_status pino_mlp_free(pino_mlp *m);

/* Network inputs and training target for one item of a context (any
 * precision): x [n][4] (device), w [n] (device, may be NULL) = 1/(l1 D_c)
 * from the full FP64 solve of the context's collapse condition (EdS or,
 * for PINO_CLASSIC_LCDM contexts, LCDM time coefficients), or 0 where the
 * particle never collapses or the network is not consulted
 * (l1 < 0.1 max|l|).  omega_m comes from the
 * item's growth table.  At most 2^28 particles per call (PINO_ERR_ARG
 * otherwise). */
pino_status pino_collapse_features(pino_ctx *ctx, const pino_item *item, float *x, float *w, void *hip_stream);

/* The BF16-MFMA network of a PINO_SURROGATE context on given inputs
 * x [n][4] -> y [n] (device), the arithmetic the collapse kernel uses. */
pino_status pino_collapse_predict(pino_ctx *ctx, const float *x, float *y, int64_t n, void *hip_stream);

/* Counts since init (or the last reset) of a PINO_SURROGATE context, one
 * per particle and radius: certified (the Newton-certified prediction was
 * accepted); fallback (consulted but not certified: full solve);
 * gated_solved (0 < l1 < 0.1 |l3|, not consulted: full solve); gated_zero
 * (l1 <= 0: F = 0 exactly, no solve).  The four add up to the evaluations
 * made; fallback + gated_solved took the full FP64 solve.  Any pointer may
 * be NULL.  Waits for the context's device. */
pino_status pino_collapse_surrogate_stats(pino_ctx *ctx, int64_t *certified, int64_t *fallback,
                                          int64_t *gated_solved, int64_t *gated_zero, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* PINO_MLP_H */
