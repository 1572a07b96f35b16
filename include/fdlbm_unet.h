/*
 * fdlbm_unet.h -- C ABI of the learned warm start of the steady-state solve:
 * a small 3-D convolutional U-Net, trained and evaluated on the GPU with
 * hand-written kernels (bf16 MFMA convolutions with FP32 accumulation), that
 * maps a geometry (solid mask) and the flow state of a packed bed to its
 * steady mole fractions, temperature and velocity.  Its prediction only
 * initialises the fields of the lattice-Boltzmann solve (fdlbm_init_fields),
 * which then relaxes them to the steady state: the method itself decides
 * the result.  This is an addition to the paper's method (which has
 * no learned component), not a reading of it.
 *
 * Network (cube edge R, a multiple of 4, >= 16; tensors channels-last
 * [sample][z][y][x][channel]):
 *   enc1  conv 32->32, conv 32->32           at R      (ReLU after each conv)
 *   enc2  2x2x2 average pool, conv 32->64, conv 64->64        at R/2
 *   bott  pool, conv 64->160, conv 160->160                   at R/4
 *   dec2  nearest 2x upsampling, concat enc2 (224), conv 224->64, conv 64->64
 *   dec1  upsampling, concat enc1 (96), conv 96->32, conv 32->32
 *   head  conv 32->32, no activation (the first n_out channels are used)
 * Every conv is 3x3x3, stride 1, zero padding 1.  The input's first c_in
 * channels come from the caller, the rest of the 32 are zero.
 *
 * Parameters: one FP32 vector; for each of the 11 convs in the order above
 * its weights W[c_out][tap][c_in] (tap = 9 (dz+1) + 3 (dy+1) + (dx+1), the
 * input read at (z+dz, y+dy, x+dx)), then its biases [c_out].  Activations
 * and weights are rounded to bf16 for the convolutions, which accumulate in
 * FP32; the master parameters and the Adam state stay FP32.
 *
 * Memory: the caller allocates one device workspace (fdlbm_unet_workspace_
 * bytes, 256-byte aligned) and keeps it alive; the library allocates none.
 * Input, target and weight arrays passed to the calls are device pointers,
 * FP32, [sample][position][channel] with position = x + R (y + R z).  All
 * work runs on the stream given at creation.  Errors: the FDLBM_E_* codes
 * of fdlbm.h; fdlbm_unet_last_error() gives a message.
 */
#ifndef FDLBM_UNET_H
#define FDLBM_UNET_H

#include <stddef.h>
#include <stdint.h>

#include "fdlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FDLBM_UNET_CPAD 32   /* padded input and output channel count */
#define FDLBM_UNET_LAYERS 11 /* convolutions                          */

typedef struct fdlbm_unet fdlbm_unet;

/* A network for cubes of edge R and up to n_max samples per call, with
 * c_in input and n_out output channels (each 1..32). */
int fdlbm_unet_create(int R, int n_max, int c_in, int n_out, void *hip_stream, fdlbm_unet **out);
void fdlbm_unet_destroy(fdlbm_unet *u);
const char *fdlbm_unet_last_error(const fdlbm_unet *u);
int fdlbm_unet_param_count(const fdlbm_unet *u, size_t *n);
int fdlbm_unet_workspace_bytes(const fdlbm_unet *u, size_t *bytes);
int fdlbm_unet_bind_workspace(fdlbm_unet *u, void *dev_ptr, size_t bytes);

/* Parameters from / to a host FP32 vector of fdlbm_unet_param_count values
 * (layout above).  Setting them resets the Adam state.  Synchronous. */
int fdlbm_unet_set_params(fdlbm_unet *u, const float *host, size_t n);
int fdlbm_unet_get_params(fdlbm_unet *u, float *host, size_t n);

/* Prediction: x [n][R^3][c_in] -> y [n][R^3][n_out] (device). */
int fdlbm_unet_forward(fdlbm_unet *u, const float *x_dev, int n, float *y_dev);

/* Loss L = sum w (y - t)^2 / wsum over every position and output channel
 * (t, w: [n][R^3][n_out], device; wsum: the sum of w, > 0) and its gradient
 * with respect to the parameters, copied to grad_host (param_count floats)
 * if not NULL.  Synchronous. */
int fdlbm_unet_gradient(fdlbm_unet *u, const float *x_dev, const float *t_dev, const float *w_dev, int n,
                        double wsum, double *loss, float *grad_host);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on that loss;
 * *loss (if not NULL) is the loss before the step (then synchronous). */
int fdlbm_unet_train_step(fdlbm_unet *u, const float *x_dev, const float *t_dev, const float *w_dev, int n,
                          double wsum, float lr, double *loss);

#ifdef __cplusplus
}
#endif
#endif
