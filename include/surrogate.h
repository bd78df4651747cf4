/* surrogate.h -- C ABI of the learned surrogate of the CSPH-TVD step on one
 * MI355X (gfx950): a stack of 3x3 convolutions that predicts the change of
 * (h, hu, hv, b) over k steps of the solver from (h, hu, hv, b, wet mask),
 * run with BF16 weights and activations on the matrix cores (FP32
 * accumulation), trained on the GPU (FP32 master weights, Adam), and applied
 * to a solver with a mass check and a fall back to the plain step.
 *
 * Network: layers l = 0..L-1, y_l = conv3x3(x_l, W_l) + b_l with zero
 * padding, ReLU after every layer but the last.  Widths channels[0..L]:
 * channels[0] = 5 inputs, channels[L] = 4 outputs, hidden widths at most 48.
 * Parameters as one FP32 vector: for each layer W_l[c_out][c_in][3][3] (row
 * major) followed by b_l[c_out].
 *
 * Errors: the SW_* codes of csph.h (SW_ERR_ARG for bad arguments, SW_ERR_HIP
 * for a failed HIP call); sws_last_error gives the text.  All calls are
 * stream-ordered on the stream given at creation; the ones returning values
 * to the host synchronise it.  Host arrays (SW_PTR_HOST) pass through a
 * pinned staging buffer the net owns and are copied synchronously.
 */
#ifndef CSPH_SURROGATE_H
#define CSPH_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "csph.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sws_net sws_net;

/* Create a network with L = nlayers layers of widths channels[0..L]
 * (channels[0] == 5, channels[L] == 4, 1 <= every width <= 48, L >= 2).
 * hip_stream: a hipStream_t (NULL: the null stream).  Parameters start at 0. */
int sws_create(const int32_t *channels, int32_t nlayers, void *hip_stream, sws_net **out);
int sws_destroy(sws_net *net);

/* Number of FP32 parameters (weights and biases of all layers). */
int sws_param_count(const sws_net *net, int64_t *n);

/* Copy the FP32 parameter vector in or out (ptr_kind: SW_PTR_HOST or
 * SW_PTR_DEVICE); setting parameters also clears the Adam moments. */
int sws_set_params(sws_net *net, const float *params, int ptr_kind);
int sws_get_params(sws_net *net, float *params, int ptr_kind);

/* Scales of the network's inputs and outputs: the network sees
 * x_c = in_scale[c] * field_c for (h, hu, hv, b) and the wet mask (c = 4,
 * 1 where h > 0), and its output o_c stands for the change
 * delta_c = out_scale[c] * o_c of (h, hu, hv, b). */
int sws_set_scales(sws_net *net, const float in_scale[5], const float out_scale[4]);

/* Network output for nimg images: x planar FP32 [nimg][5][ny][nx] (already
 * scaled network inputs), y planar FP32 [nimg][4][ny][nx].  Rows are dense
 * (no pitch). */
int sws_forward(sws_net *net, const float *x, float *y, int32_t nimg, int32_t nx, int32_t ny,
                int ptr_kind);

/* Gradient of the loss (as in sws_train_step) with respect to every
 * parameter, without an update: grad receives the FP32 vector in parameter
 * order (ptr_kind as for the inputs); *loss (may be NULL) the loss.
 * Synchronises.  Training calls (sws_grad, sws_train_step, sws_train) take
 * images of nx * 96 < 2^31 (one row of 48 BF16 channels must fit a 31-bit
 * byte count); wider images are SW_ERR_ARG before any device work. */
int sws_grad(sws_net *net, const float *x, const float *target, int32_t nimg, int32_t nx,
             int32_t ny, float *grad, double *loss, int ptr_kind);

/* One training step on nimg images: forward, loss = mean over all outputs of
 * (y - target)^2, backward, one Adam update of every parameter (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected; the step count is kept by the net).
 * *loss (may be NULL) receives the loss before the update (synchronises). */
int sws_train_step(sws_net *net, const float *x, const float *target, int32_t nimg, int32_t nx,
                   int32_t ny, float lr, double *loss, int ptr_kind);

/* Advance a solver by k steps with the surrogate: the predicted change is
 * added to the solver's state (depth clamped at 0, momentum zeroed where the
 * depth is 0) unless the relative change of the water volume or of the bed
 * sum exceeds max_drift (closed domains: neither may change), in which case
 * the solver takes the k steps itself with fixed step dt.  Either way the
 * model time advances by k dt.  *used (may be NULL) receives 1 if the
 * surrogate's prediction was kept.  One call of sws_advance_K without
 * residual checks.  Synchronises. */
int sws_advance(sws_net *net, sw_ctx *solver, int32_t k, double dt, double max_drift,
                int32_t *used);

/* Training run on the GPU (the loop the paper's solver-generated data feeds;
 * the learning part of the method is this project's, as the paper has none):
 * npairs pairs of already scaled inputs x [npairs][5][ny][nx] and scaled
 * targets [npairs][4][ny][nx] (host or device, per ptr_kind) are copied to the
 * device once; each of cfg->steps Adam steps (sws_train_step) takes cfg->batch
 * distinct pairs drawn with SplitMix64 from cfg->seed, with the learning rate
 * cfg->lr 0.5 (1 + cos(pi step / steps)).  *report (may be NULL): the first
 * step's loss and the mean of the last min(50, steps); losses (host, may be
 * NULL): every step's loss (reading them synchronises every step).
 * Allocates and frees a device copy of the set; synchronises. */
typedef struct {
    int32_t steps;
    int32_t batch;
    float lr;
    uint64_t seed;
} sws_train_cfg;
typedef struct {
    double first_loss, final_loss;
    int32_t steps;
} sws_train_report;
int sws_train(sws_net *net, const float *x, const float *target, int32_t npairs, int32_t nx,
              int32_t ny, const sws_train_cfg *cfg, sws_train_report *report, float *losses,
              int ptr_kind);

/* n_calls surrogate calls of k steps each on a solver (sws_advance's step,
 * called again and again), with the checks that decide whether a prediction
 * is kept:
 *  - conservation: the relative change of the water volume, and of the bed
 *    volume sum b, must stay within max_drift (a closed domain without
 *    sources); else the solver takes the k plain steps (fixed dt);
 *  - residual (every check_every-th call, 0 = never): the plain solver takes
 *    the same k steps from the same state and judges the prediction: if the
 *    largest depth difference exceeds max_err (m), the plain result is kept;
 *  - stability: the prediction must admit the step dt by Eq. 7
 *    (sw_step_bound), so the solver can go on from it; else the state of the
 *    call's start is restored and the solver takes the k plain steps.
 * The model time advances by k dt per call either way.  *stats (may be NULL)
 * receives the counts and the largest drift and residual seen.
 * Synchronises. */
typedef struct {
    int32_t calls;               /* surrogate calls made */
    int32_t kept;                /* predictions installed */
    int32_t fallbacks_volume;    /* calls the conservation check sent to the plain step */
    int32_t fallbacks_residual;  /* checked calls whose depth residual exceeded max_err */
    int32_t checks;              /* calls the plain step judged */
    double max_volume_drift;     /* largest relative water or bed volume change predicted */
    double max_residual;         /* largest depth difference (m) at a check */
    int32_t fallbacks_stability; /* predictions whose Eq. 7 step bound was below dt */
} sws_stats;
int sws_advance_K(sws_net *net, sw_ctx *solver, int32_t n_calls, int32_t k, double dt,
                  double max_drift, int32_t check_every, double max_err, sws_stats *stats);

/* Text of the last error on net (never NULL). */
const char *sws_last_error(const sws_net *net);

#ifdef __cplusplus
}
#endif

#endif
