/*
 * rod_surrogate.h -- C boundary of the learned coarse step.
 *
 * The surrogate is this build's addition to the discrete Cosserat-rod step
 * (the paper, Elastica++, only motivates learning-oriented workflows in its
 * introduction): a per-element MLP that maps a 5-element stencil window of a
 * rod, expressed in the centre element's material frame, to the change of
 * that element's node and director state over k plain substeps.  Network:
 * 96 inputs -> 256 -> 256 -> 256 -> 12 outputs, SiLU after the first three
 * layers, BF16 weights and activations, FP32 accumulation (MFMA), FP32 bias
 * and output; FP32 master weights trained with Adam.
 *
 * Conventions are those of rod.h: 0 or a negative ROD_E* code,
 * rod_last_error() for the message, asynchronous on `stream` unless stated.
 * Parameter vectors use the layer-major layout: for each layer W [K][N]
 * row-major then b [N], layers (96,256), (256,256), (256,256), (256,12);
 * ROD_SURROGATE_PARAMS values in all.
 */
#ifndef ROD_SURROGATE_H
#define ROD_SURROGATE_H

#include <stdint.h>

#include "rod.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ROD_SURROGATE_INPUTS 96
#define ROD_SURROGATE_OUTPUTS 12
#define ROD_SURROGATE_PARAMS 159500

typedef struct rod_surrogate rod_surrogate;

typedef struct {
    int32_t k_substeps;      /* plain substeps replaced by one coarse step (> 0) */
    uint64_t seed;           /* weight initialisation: W ~ U(-a, a), a = sqrt(6 / fan_in), b = 0 */
    int32_t max_rows;        /* rows per MLP workspace chunk; 0: 65536 */
} rod_surrogate_desc;

/* Allocate the network, its Adam state and workspace on the current device.
 * ROD_EINVAL for k_substeps <= 0 or max_rows < 0 (or not a multiple of 64). */
int rod_surrogate_create(const rod_surrogate_desc *desc, rod_surrogate **out);
void rod_surrogate_destroy(rod_surrogate *s);

/* Copy FP32 master weights in (host, ROD_SURROGATE_PARAMS values, layout
 * above; resets Adam) or out.  Synchronous. */
int rod_surrogate_set_params(rod_surrogate *s, const float *params);
int rod_surrogate_get_params(rod_surrogate *s, float *params);

/* Raw network on device buffers: x BF16 [M][96] (row-major), y FP32 [M][12]. */
int rod_surrogate_forward(rod_surrogate *s, const void *x_bf16, int64_t M, float *y, void *stream);

/* Mean squared error of y = net(x) against t (FP32 [M][12], device) over the
 * entries where mask (FP32 [M][12], device, or NULL = all) is 1, and its
 * gradient with respect to every parameter, written to host `grads`
 * (ROD_SURROGATE_PARAMS values) and `*loss`.  M <= max_rows, M a multiple
 * of 32.  Synchronises `stream`. */
int rod_surrogate_gradients(rod_surrogate *s, const void *x_bf16, const float *t, const float *mask,
                            int64_t M, float *grads, float *loss, void *stream);

/* One Adam step (b1 0.9, b2 0.999, eps 1e-8) at learning rate lr on the
 * gradient of the same loss; *loss (host, may be NULL) receives the loss
 * before the step.  Synchronises `stream` when loss is not NULL. */
int rod_surrogate_train_step(rod_surrogate *s, const void *x_bf16, const float *t, const float *mask,
                             int64_t M, float lr, float *loss, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ROD_SURROGATE_H */
