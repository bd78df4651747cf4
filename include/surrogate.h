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
 * Synchronises. */
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
 * depth is 0) unless the relative change of the water volume exceeds
 * max_drift (closed domains: the volume must not change), in which case the
 * solver takes the k steps itself with fixed step dt.  Either way the model
 * time advances by k dt.  *used (may be NULL) receives 1 if the surrogate's
 * prediction was kept.  Synchronises. */
int sws_advance(sws_net *net, sw_ctx *solver, int32_t k, double dt, double max_drift,
                int32_t *used);

/* Text of the last error on net (never NULL). */
const char *sws_last_error(const sws_net *net);

#ifdef __cplusplus
}
#endif

#endif
