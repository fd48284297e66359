/*
 * lbm_nn.h - C ABI of the learned warm start: a 3D convolutional
 * encoder-decoder that maps the Rayleigh number of the differentially
 * heated cavity (Sec. 3 of arXiv:1710.04751) and the cell coordinates to
 * the steady fields (u, v, w, T), trained on steady states that the
 * library's own solver produces, and used to initialise that solver
 * (lbm_init_macros).  The network is not part of the paper: it shortens the
 * time the paper's method takes to reach the steady state it reports.
 *
 * Arithmetic: BF16 weights and activations, FP32 accumulation in the gfx950
 * matrix cores (MFMA), FP32 master weights, gradients and Adam moments.
 *
 * Network (levels of 16, 32, 64, 128 channels on grids G, G/2, G/4, G/8):
 *   enc1a 4->16, enc1b 16->16 | avg-pool | enc2a 16->32, enc2b 32->32 |
 *   avg-pool | enc3a 32->64, enc3b 64->64 | avg-pool | bota 64->128,
 *   botb 128->128, botc 128->128 | upsample, concat [enc3b, up] |
 *   dec3a 192->64, dec3b 64->64 | upsample, concat [enc2b, up] |
 *   dec2a 96->32, dec2b 32->32 | upsample, concat [enc1b, up] |
 *   dec1a 48->16, dec1b 16->16 | head 16->4 (1x1x1, linear).
 * Every 3x3x3 convolution (zero padding, cross-correlation) is followed by
 * ReLU; pooling averages 2x2x2 blocks, upsampling repeats each cell 2x2x2.
 * Input channels: (log10 Ra - 4) / 2 and the cell-centre coordinates
 * 2 (i + 1/2) / G - 1 along x, y, z.  Output channels: u, v, w, T in the
 * units of the training targets (see target_scale).
 *
 * Parameter vector (FP32, device): layer after layer in the order above,
 * the weight w[co][kz][ky][kx][ci] then the bias b[co]; 1,903,428 values.
 *
 * Tensors: activations are channels-last BF16, x[n][z][y][x][c] with x
 * fastest; the network output and the targets are channel-first FP32,
 * out[n][c][z][y][x] (the layout of lbm_macros / lbm_init_macros fields).
 *
 * Conventions as in lbm.h: every function returns an lbm_status, device
 * memory is the caller's, work goes on the stream given at creation, only
 * functions documented as synchronising wait for the device.
 */
#ifndef LBM_NN_H_
#define LBM_NN_H_

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_nn lbm_nn;

typedef struct lbm_nn_config {
    int32_t grid;          /* edge G of the cubic grid: a power of two, 8..256 */
    int32_t batch;         /* most samples per call (1..64) */
    float lr;              /* Adam step size */
    float beta1, beta2;    /* Adam moment decay rates (0.9, 0.999) */
    float eps;             /* Adam denominator guard (1e-8) */
    float target_scale[4]; /* the loss compares output channel c with
                              target channel c times target_scale[c] */
} lbm_nn_config;

/* Number of parameters of the network (1,903,428). */
int64_t lbm_nn_param_count(void);

/* Bytes of device workspace for a configuration; 0 if it is invalid. */
size_t lbm_nn_workspace_bytes(const lbm_nn_config* c);

/* Create over caller device memory (256-byte aligned, borrowed until
 * lbm_nn_destroy).  Parameters start at zero: set them with
 * lbm_nn_set_params. */
lbm_status lbm_nn_create(const lbm_nn_config* c, void* workspace, size_t bytes, void* stream,
                         lbm_nn** out);
lbm_status lbm_nn_destroy(lbm_nn* nn);

/* Copy the FP32 parameter vector in (device pointer) and reset the Adam
 * moments and step count; or copy it out.  Asynchronous. */
lbm_status lbm_nn_set_params(lbm_nn* nn, const float* params);
lbm_status lbm_nn_get_params(lbm_nn* nn, float* params);

/* Forward pass for n samples with Rayleigh numbers given as log10 Ra (host
 * array of n): out (device, FP32, [n][4][G][G][G]) = network output times
 * out_scale[c] (host array of 4; NULL means 1).  Asynchronous. */
lbm_status lbm_nn_forward(lbm_nn* nn, int32_t n, const float* log10_ra, float* out,
                          const float* out_scale);

/* Loss and gradient without a parameter update: targets (device, FP32)
 * hold target_count samples of [4][G][G][G] values target_stride floats
 * apart (target_stride >= 4 G^3); sample i of the call uses
 * targets[target_index[i]] (host array of n).  An index outside
 * [0, target_count) is LBM_ERR_ARG before any launch.  Loss = mean over
 * n * 4 * G^3 of (output - target * target_scale)^2.  grad (device, FP32,
 * parameter layout) receives the gradient when not NULL; *loss (host) the
 * loss.  Synchronises. */
lbm_status lbm_nn_gradient(lbm_nn* nn, int32_t n, const float* log10_ra, const float* targets,
                           int64_t target_count, const int32_t* target_index,
                           int64_t target_stride, float* grad, double* loss);

/* One training step: forward, loss, backward and an Adam update of every
 * parameter, on the same arguments as lbm_nn_gradient.  loss (host) may be
 * NULL; when given the call synchronises to return it. */
lbm_status lbm_nn_train_step(lbm_nn* nn, int32_t n, const float* log10_ra,
                             const float* targets, int64_t target_count,
                             const int32_t* target_index, int64_t target_stride, double* loss);

/* Change the Adam step size for later training steps (learning-rate
 * schedules); lr > 0. */
lbm_status lbm_nn_set_lr(lbm_nn* nn, float lr);

/* Output of layer `layer` (0..15 in the order above; 15 is the head,
 * before out_scale) of the last forward pass as FP32 (device), channels-
 * last [n][g][g][g][c] on that layer's grid g; for checking the kernels.
 * The head's output is computed on this call from its input of that pass
 * with the current parameters (after lbm_nn_train_step: the updated ones).
 * n must equal the sample count of that pass (LBM_ERR_ARG otherwise). */
lbm_status lbm_nn_activation(lbm_nn* nn, int32_t layer, int32_t n, float* out);

/* Algorithmic floating-point operations of one forward pass and of one
 * training step (forward + backward) for n samples (2 per multiply-add). */
lbm_status lbm_nn_flops(const lbm_nn* nn, int32_t n, double* forward, double* train_step);

#ifdef __cplusplus
}
#endif

#endif /* LBM_NN_H_ */
