/*
 * rod_surrogate.h -- C boundary of the learned coarse step.
 *
 * The surrogate is this library's addition to the discrete Cosserat-rod step
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

/*
 * Windows and the data path (FP32 batches only: ROD_EUNSUPPORTED otherwise).
 * A rod of n elements has n + 1 windows, rod-major: window w < n is centred on
 * element w and targets node w and element w; window n is centred on element
 * n - 1 and targets node n.  With tau = k dt and lh_c the centre element's
 * rest length, everything in the centre element's frame Q_c:
 *   96 features = 5 stencil slots (elements c-2..c+2) x 16
 *     [Q_c (x_j - x_c)/lh_c, Q_c (u_j - u_c) tau/lh_c, rows 0-1 of Q_j Q_c^T,
 *      omega_j tau, 1]   (x midpoint, u mean node velocity; zeros off the rod)
 *   + 16 globals [Q_c v_p tau/lh_c, Q_c (r_p - x_c)/lh_c, log10(E/1e6),
 *      radius/lh_c, log10(tau/T_b) with T_b = lh_c^2 sqrt(rho A/(E I)),
 *      alpha_c, clamped-base flag, c/n, end flag, couple amplitude / 1e-5,
 *      sin and cos of the couple phase];
 *   12 targets, the departures from free flight over tau (constant node
 *      velocity and element angular velocity) = [Q_c (dr_p - v_p tau)/lh_c,
 *      Q_c dv_p tau/lh_c, theta - omega_c tau with Q_c(t+tau) =
 *      exp(-[theta]x) Q_c(t), d omega_c tau]; the element part of window n is
 *      masked.  Applying deltas adds the free flight back.
 */

/* Raw FP32 features [W][96] of the batch's current state (device buffer). */
int rod_surrogate_features(rod_surrogate *s, rod_batch *b, float *features, void *stream);

/* Training sample at the current state: features [W][96], then k plain steps
 * of the batch (rod_step), then targets [W][12] and the loss mask [W][12]
 * (device buffers). */
int rod_surrogate_collect(rod_surrogate *s, rod_batch *b, float *features, float *targets, float *mask,
                          void *stream);

/* Perturb the free part of the batch state in place (seeded, counter-based
 * N(0, 1) deviates g): node positions by noise[0] lh g, node velocities by
 * noise[1] lh / tau g, director frames by exp(-[noise[2] g]x), angular
 * velocities by noise[3] / tau g, with lh the rest length of the node's own
 * element (element n-1 for node n).  Clamped nodes and elements are left
 * alone.  The same (seed, batch) gives the same perturbation. */
int rod_surrogate_perturb(rod_surrogate *s, rod_batch *b, const float *noise, uint64_t seed, void *stream);

/* As rod_surrogate_collect, but the features are those of the perturbed state
 * (rod_surrogate_perturb with noise and seed) while the batch steps on from
 * the unperturbed state, and the targets lead from the perturbed state to the
 * plain result: the network learns to return to the trajectory. */
int rod_surrogate_collect_noisy(rod_surrogate *s, rod_batch *b, const float *noise, uint64_t seed, float *features,
                                float *targets, float *mask, void *stream);

/* Apply raw deltas [W][12] (device) to the batch as one coarse step and
 * advance its clock by k steps: free flight plus the deltas, then each
 * rotated director frame is moved to its nearest rotation (one Newton-Schulz
 * polar step).  Clamped ends are left unchanged. */
int rod_surrogate_apply(rod_surrogate *s, rod_batch *b, const float *deltas, void *stream);

/* Standardisation of inputs and outputs (host arrays: 96, 96, 12, 12 values;
 * standard deviations > 0): the network sees (x - mu_x)/sd_x and predicts
 * (t - mu_t)/sd_t. */
int rod_surrogate_set_normalization(rod_surrogate *s, const float *mu_x, const float *sd_x, const float *mu_t,
                                    const float *sd_t);
int rod_surrogate_get_normalization(rod_surrogate *s, float *mu_x, float *sd_x, float *mu_t, float *sd_t);

typedef struct {
    int32_t warmup_steps;    /* plain steps before the first sample */
    int32_t n_samples;       /* collect() calls; all windows of the batch each time */
    int32_t sample_stride;   /* plain steps from one sample's start to the next (>= k) */
    int32_t epochs;
    int32_t batch_rows;      /* minibatch rows: a multiple of 64, <= max_rows */
    float lr;                /* peak learning rate, cosine decay to lr_min over all steps */
    float lr_min;
    float val_fraction;      /* share of windows held out for validation */
    uint64_t seed;           /* shuffling and perturbations */
    float noise[4];          /* perturbation levels (rod_surrogate_perturb); sample i uses
                                (i mod 4) / 3 of them, so a quarter of the samples is clean */
} rod_train_desc;

/* Generate trajectories with the plain integrator on `b` (advancing it),
 * standardise, and train the network with Adam on minibatches.  Host
 * outputs: epoch_loss[epochs] (mean training loss per epoch, may be NULL) and
 * *val_loss (loss on the held-out windows after training, may be NULL).
 * Synchronises `stream`. */
int rod_surrogate_train(rod_surrogate *s, rod_batch *b, const rod_train_desc *d, float *epoch_loss,
                        float *val_loss, void *stream);

/*
 * The learned coarse step with the plain integrator as judge and fallback.
 * Each coarse step: features of every window, the network, and the predicted
 * deltas applied to every rod not on the plain step (the clock advances by
 * k steps); rods on the plain step take k plain steps instead.  Every
 * judge_every coarse steps a seeded sample of judge_fraction of the rods
 * (at least one) that are still on the coarse step is re-run by the plain
 * integrator from the state saved at the start of the window; a sampled rod
 * whose max_j |r_j - r_j(plain)| / L exceeds max_pos_error, whose
 * max |Q Q^T - I| exceeds max_orth_error, or whose strain energy (shear plus
 * bending, as rod_energy) differs from the plain re-run's by more than
 * max_energy_error times the re-run's mechanical energy (kinetic plus strain)
 * takes the plain state and stays on the plain step.  Non-finite errors fail.
 * Requires an FP32 batch whose rods all have the same element count
 * (ROD_EUNSUPPORTED otherwise).  The fallback flags belong to the last batch
 * this handle worked on: using the handle with another batch resets them.
 * Synchronises `stream` at the end of every judge window.
 */
typedef struct {
    int32_t judge_every;     /* coarse steps per judge window (> 0) */
    float judge_fraction;    /* in (0, 1] */
    float max_pos_error;     /* relative to the rod's rest length */
    float max_orth_error;
    uint64_t seed;
    float max_energy_error;  /* relative strain-energy difference */
} rod_judge_desc;

typedef struct {
    int64_t coarse_steps;    /* taken by this call */
    int64_t judge_windows;
    int64_t rods_judged;
    int64_t rods_failed;     /* sent to the plain step by this call */
    int64_t rods_plain;      /* on the plain step after the call */
    double max_pos_error;    /* largest judged errors of this call */
    double max_orth_error;
    double max_energy_error;
} rod_surrogate_stats;

int rod_surrogate_step(rod_surrogate *s, rod_batch *b, int64_t n_coarse, const rod_judge_desc *j,
                       rod_surrogate_stats *stats, void *stream);

/* Write the network (FP32 parameters, normalisation, k) to a file, or read
 * one back (resets Adam).  ROD_EINVAL when the file cannot be opened, is not
 * a file of this network, or was written for another k.  Synchronous. */
int rod_surrogate_save(rod_surrogate *s, const char *path);
int rod_surrogate_load(rod_surrogate *s, const char *path);

/* Per-rod fallback flags of the batch (host int32 [R], 1 = on the plain
 * step); reset puts every rod back on the coarse step. */
int rod_surrogate_fallback_flags(rod_surrogate *s, rod_batch *b, int32_t *flags);
int rod_surrogate_reset_fallback(rod_surrogate *s, rod_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* ROD_SURROGATE_H */
