/*
 * fftlb_cnn.h: C ABI of the warm-start network of the FFT-LB solver (gfx950).
 *
 * A small convolutional encoder-decoder maps the normalised initial fields of a run
 * (rho0 / rho_c, T0 / T_c, T_target / T_c) on a periodic h x w grid to near-equilibrium
 * (rho, T); fftlb_init then starts the FFT-LB run from f^eq of the prediction, and the run
 * itself decides when equilibrium is reached (the prediction only shortens the way).  The
 * network is not part of the paper's method; it is trained on relaxed fields the solver
 * produced.
 *
 * Network (every convolution 3 x 3, periodic padding, cross-correlation
 * conv(X)[co, y, x] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] X[ci, y + ky - 1, x + kx - 1]):
 *   1: 3 -> 32, stride 1         2: 32 -> 32, stride 2 (output (y, x) centred on input (2y, 2x))
 *   3: 32 -> 32, stride 2        4: nearest upsampling by 2, 32 -> 32, stride 1
 *   5: upsampling by 2, 32 -> 32 6: 32 -> 2, stride 1, linear
 *   GELU z Phi(z) after layers 1-5; output = input channels 0, 1 + layer-6 output.
 * Parameters: one float vector of FFTLB_CNN_PARAMS entries, per layer W[Cout][Cin][3][3]
 * followed by b[Cout].
 *
 * Arithmetic: every convolution, forward and backward, runs on the bf16 matrix cores with
 * FP32 accumulation (operands rounded to bf16 to nearest even on the way in); activations,
 * parameters, gradients and Adam state are FP32.  The weight gradient is summed over
 * pixel chunks in a fixed order, so training is deterministic.  Loss: mean squared error over all output
 * values.  Adam: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected.
 *
 * Conventions as in fftlb.h: device pointers, caller-owned workspace, asynchronous on
 * `stream`, FFTLB_OK or a negative FFTLB_E* code.  Tensors are [n][c][h][w] float32.
 */
#ifndef FFTLB_CNN_H
#define FFTLB_CNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFTLB_CNN_PARAMS 38466

typedef struct fftlb_cnn fftlb_cnn;

/* Workspace for batches of up to max_batch samples of h x w (h, w multiples of 4, >= 8). */
int fftlb_cnn_workspace_bytes(int32_t h, int32_t w, int32_t max_batch, size_t* bytes);

/* Create a network on `workspace` with initial parameters `params` (device, copied). */
int fftlb_cnn_create(int32_t h, int32_t w, int32_t max_batch, void* workspace, size_t ws_bytes,
                     const float* params, void* stream, fftlb_cnn** out);

/* Forward pass of n samples x [n][3][h][w]; y [n][2][h][w] (may be NULL: the output
 * stays in the network's buffer, see fftlb_cnn_read_buffer). */
int fftlb_cnn_forward(fftlb_cnn* c, const float* x, float* y, int32_t n, void* stream);

/* Forward and backward pass against target [n][2][h][w]: the gradient of the loss is
 * kept for fftlb_cnn_adam_step and copied to grad (device, FFTLB_CNN_PARAMS, or NULL);
 * the loss goes to *loss (device double, or NULL). */
int fftlb_cnn_gradient(fftlb_cnn* c, const float* x, const float* target, int32_t n, float* grad,
                       double* loss, void* stream);

/* One Adam update of the parameters with the last gradient, learning rate lr > 0. */
int fftlb_cnn_adam_step(fftlb_cnn* c, float lr, void* stream);

/* Copy the parameters out / in (set_params also resets the Adam state). */
int fftlb_cnn_get_params(const fftlb_cnn* c, float* params, void* stream);
int fftlb_cnn_set_params(fftlb_cnn* c, const float* params, void* stream);

/* Copy `count` floats of an internal buffer of the last call into dst (device), layer
 * 1..6: kind 0 = pre-activation Z [n][Cout][H][W] of the layer, 1 = dL/dZ (after
 * fftlb_cnn_gradient), 2 = the layer's output (GELU(Z); for layer 6 the network output).
 * count may not exceed the buffer (max_batch samples). */
int fftlb_cnn_read_buffer(const fftlb_cnn* c, int32_t layer, int32_t kind, float* dst, size_t count,
                          void* stream);

/* Warm-start transform of a prediction into the initial fields of a run (the network is
 * not part of the paper; this prepares its output for fftlb_init).  pred: device [2][h][w],
 * the predicted rho / rho_c and T / T_c; rho0: device [h][w], the run's initial density (its
 * total is the mass to keep).  Writes device [h][w] rho_out and T_out:
 *   1. rho = clip(rho_c pred_0, 1e-3 rho_c, rho_max) (rho_max < 1/b keeps the pressure of
 *      Eq. (18) finite; rho_max > 1e-3 rho_c);
 *   2. one pass of the periodic binomial filter (1 2 1)/4 along x, then y (it removes the
 *      grid-scale content, which the windowed derivatives barely move);
 *   3. the mass deficit M0 - M (M0 = sum rho0) added in proportion to the interface weight
 *      w = |grad rho| (periodic central differences), so the bulk densities stay (a field
 *      with sum w <= 1e-6 M is rescaled instead); clipped again; rescaled to the exact M0;
 *   4. T uniform at the mean of T_c pred_1, at least 1e-2 T_c.
 * Sums are FP64 in a fixed order (deterministic).  The total energy is matched afterwards on
 * the solver (fftlb_match_energy).  Uses the network's input buffer as scratch. */
int fftlb_cnn_project(fftlb_cnn* c, const float* pred, const float* rho0, float rho_c, float T_c, float rho_max,
                      float* rho_out, float* T_out, void* stream);

/* Warm start of one run: the network's prediction from the initial fields rho0, T0 (device
 * [h][w]) and the run's temperature T_target (input channels rho0 / rho_c, T0 / T_c,
 * T_target / T_c), then fftlb_cnn_project of that prediction into rho_out, T_out. */
int fftlb_cnn_warm_start(fftlb_cnn* c, const float* rho0, const float* T0, float T_target, float rho_c,
                         float T_c, float rho_max, float* rho_out, float* T_out, void* stream);

/* Release the handle (the workspace is untouched). */
int fftlb_cnn_destroy(fftlb_cnn* c);

#ifdef __cplusplus
}
#endif
#endif /* FFTLB_CNN_H */
