/* Convolutional surrogate of the two-fluid active-nematic solver: C ABI.
 *
 * The network advances the solver state x = (phi, Qxx, Qxy, u_a,x, u_a,y,
 * u_p,x, u_p,y) (the fields of the Model section) by k lattice steps, to
 * fast-forward the coarsening the Results section follows.  Architecture: six
 * periodic 3x3 convolutions 7 -> 48 -> 48 -> 48 -> 48 -> 48 -> 7 with SiLU after
 * the first five, acting on x / s_in (fixed per-channel input scales); the
 * output y is the increment in units of per-channel output scales s_out,
 * prediction = x + s_out * y.  Training loss: the mean over samples, channels
 * and sites of (y - (x_target - x) / s_out)^2; optimiser Adam.
 *
 * Precision: weights, activations and back-propagated gradients are bfloat16
 * (round to nearest even), products accumulate in fp32 on the matrix cores; the
 * master parameters, Adam moments, pre-activations and the output are fp32; loss
 * and comparison sums are fp64.
 *
 * Parameter vector (fp32, host): layer by layer, W[co][ci][3][3] (tap (dy, dx)
 * reads the site (y + dy - 1, x + dx - 1)) then b[co].
 *
 * State arrays passed to the network are device fp32 [B][7][ny][nx] (x fastest),
 * or stacks of such samples; ny and nx must be multiples of 16.  All device work
 * is enqueued on the handle's stream; functions that return a host result
 * synchronise it.  Return codes are those of tfan.h (0 = success).
 */
#ifndef TFAN_CNN_H
#define TFAN_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "tfan.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfan_cnn tfan_cnn;

/* Number of fp32 parameters of the network (89,239). */
int64_t tfan_cnn_param_count(void);

/* Device workspace for batches of `batch` samples on ny x nx grids; train != 0
 * reserves the activations and gradients of the backward pass.  0 if the sizes
 * are invalid (batch < 1, ny or nx not a positive multiple of 16, more than 2^28
 * sites per batch). */
size_t tfan_cnn_workspace_bytes(int32_t batch, int32_t ny, int32_t nx, int32_t train);

/* Creates a network bound to `hip_stream` (NULL = default stream) using the
 * caller's device workspace (256-byte aligned, at least the size above; the
 * caller keeps ownership and must keep it alive until tfan_cnn_destroy).
 * Parameters start at zero; scales at 1.  TFAN_EINVAL / TFAN_ENOMEM /
 * TFAN_EHIP. */
int tfan_cnn_create(int32_t batch, int32_t ny, int32_t nx, int32_t train, void* dev_workspace, size_t bytes,
                    void* hip_stream, tfan_cnn** out);

/* Parameters (host fp32, tfan_cnn_param_count() values).  Setting them also
 * resets the Adam moments and step count. */
int tfan_cnn_set_params(tfan_cnn* c, const float* params);
int tfan_cnn_get_params(tfan_cnn* c, float* params);

/* Per-channel input scales s_in[7] and output scales s_out[7] (> 0, finite). */
int tfan_cnn_set_scales(tfan_cnn* c, const float* s_in, const float* s_out);

/* Prediction x + s_out * y for the batch x_dev [B][7][ny][nx] into out_dev (same
 * shape; may not alias x_dev).  Asynchronous. */
int tfan_cnn_forward(tfan_cnn* c, const float* x_dev, float* out_dev);

/* Loss and gradient for the batch made of samples idx[0..B-1] of the stacks
 * x_dev and target_dev (sample i at offset i * 7 * ny * nx).  grads (host,
 * param_count values) and loss may be NULL; when either is given the call
 * synchronises.  Requires a network created with train != 0. */
int tfan_cnn_gradients(tfan_cnn* c, const float* x_dev, const float* target_dev, int64_t samples,
                       const int32_t* idx, float* grads, double* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * gradient of the same batch; loss (may be NULL: then no synchronisation)
 * receives the loss before the update. */
int tfan_cnn_train_step(tfan_cnn* c, const float* x_dev, const float* target_dev, int64_t samples,
                        const int32_t* idx, float lr, double* loss);

/* Per-channel sums over a batch of [B][7][ny][nx] arrays: out[2c] = sum (a - b)^2,
 * out[2c + 1] = sum b^2 (fp64; synchronises). */
int tfan_cnn_compare(tfan_cnn* c, const float* a_dev, const float* b_dev, double* out);

int tfan_cnn_sync(tfan_cnn* c);
void tfan_cnn_destroy(tfan_cnn* c);
/* Message of the last failure of c (or of a failed create when c is NULL). */
const char* tfan_cnn_last_error(const tfan_cnn* c);

#ifdef __cplusplus
}
#endif
#endif
