/*
 * fftlb.h: C ABI of the MI355X (gfx950) FFT-LB solver for thermal liquid-vapour systems.
 *
 * The library advances the 33 discrete-velocity distributions f_ki of the
 * Watari-Tsutahara thermal model with the Gonnella-Lamura-Sofonea van der Waals
 * force (Gan, Xu, Zhang, Li, "FFT-LB modeling of thermal liquid-vapor systems"):
 *
 *   f^{n+1} = f^n - dt v.grad f^n - (dt/tau)(f^n - f^eq) + dt I        (Sec. 3, Eq. (24) form)
 *
 * on a periodic nx x ny grid, with every spatial derivative (the convection term
 * and the derivatives inside the force, Eqs. (19)-(23)) taken by the windowed FFT
 * of Sec. 3.6: forward transform, multiplication by i k_m (Eqs. (44)-(47)),
 * inverse transform.  Arithmetic is FP32; global mass, momentum and energy are
 * reduced in FP64.
 *
 * Conventions shared by every entry point
 *  - Fields are row-major [ny][nx] float32, x fastest; distributions are
 *    [33][ny][nx] with q = 0 the rest particle and q = 1 + 8(k-1) + (i-1) for speed
 *    group k = 1..4 (speeds 1.0, 1.9, 2.9, 4.3) and direction i = 1..8 (angle (i-1) pi/4),
 *    as in Eq. (1).
 *  - Every pointer argument that carries field data is a DEVICE pointer on the
 *    device current at the call.  The caller owns all device memory: the workspace,
 *    inputs and outputs.  The library never allocates or frees device memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All work is
 *    enqueued on it asynchronously; no call synchronises, except fftlb_init (it
 *    uploads small tables from host memory and waits for them) and fftlb_destroy.
 *  - Return value: FFTLB_OK (0) or a negative error code; calls never abort.
 *    Argument errors are detected on the host before any device work is enqueued.
 *  - A handle is used from one host thread at a time.
 */
#ifndef FFTLB_H
#define FFTLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFTLB_OK 0
#define FFTLB_EINVAL (-1)    /* bad configuration, size or pointer                        */
#define FFTLB_ENOSPC (-2)    /* workspace smaller than fftlb_workspace_bytes() or misaligned */
#define FFTLB_EHIP (-3)      /* HIP runtime error; fftlb_last_error() has the message      */
#define FFTLB_EUNSTABLE (-4) /* non-finite values detected (reported by fftlb_moments)     */

#define FFTLB_Q 33
#define FFTLB_NGLOBALS 8
#define FFTLB_WORKSPACE_ALIGN 256

/* Model and discretisation parameters (Sec. 2.2; the paper's values are listed in
 * its Sec. 3.5: dx = dy = 1/256, dt = 1e-5, tau = 1e-2, K = 1e-5, H = 0, zeta = 0,
 * q = -0.004, window k4; EOS a = 9/8, b = 1/3).
 *  nx, ny        grid size; each a power of two (8 <= nx <= 2048, 4 <= ny <= 2048) or
 *                3 * 2^p with 48 <= n <= 768; ny a multiple of max(1, 64 / (nx / 2)).
 *  dx, dy, dt    lattice spacings and time step, > 0.
 *  tau           BGK relaxation time, > 0; +inf switches the collision off.
 *  K, H          gradient coefficient M = K + H T of the pressure tensor (Eq. (19)), >= 0.
 *  zeta          bulk viscosity in the force (Eqs. (21), (22)).
 *  q             Prandtl-number parameter of C_q (Eq. (23)).
 *  a, b          van der Waals constants of P = rho T/(1 - b rho) - a rho^2 (Eq. (18)
 *                with the paper's 3/(3 - rho) and 9/8 written as 1/(1 - b rho) and a), >= 0.
 *  filter_order  0 = exact wavenumber k, 1..4 = windowed k_1..k_4 (Eqs. (44)-(47)). */
typedef struct fftlb_config {
  int32_t nx, ny;
  double dx, dy, dt;
  double tau, K, H, zeta, q;
  double a, b;
  int32_t filter_order;
  int32_t reserved; /* must be 0 */
} fftlb_config;

typedef struct fftlb_handle fftlb_handle;

/* Bytes of device workspace fftlb_init needs for `cfg` (about 88 * nx * ny * 4 bytes).
 * Returns FFTLB_EINVAL for an unsupported configuration. */
int fftlb_workspace_bytes(const fftlb_config* cfg, size_t* bytes);

/* Initialise a solver on `workspace` (device memory, FFTLB_WORKSPACE_ALIGN-aligned, at
 * least fftlb_workspace_bytes bytes; it must outlive the handle).  The distribution is
 * set to the local equilibrium f^eq(rho0, u0, T0) of Eq. (3); rho0, ux0, uy0, T0 are
 * device [ny][nx] float32 fields read only during the call (rho0 > 0, T0 > 0 and
 * b rho0 < 1 are the caller's responsibility).  On success *out receives a host-side
 * handle to release with fftlb_destroy. */
int fftlb_init(const fftlb_config* cfg, void* workspace, size_t ws_bytes,
               const float* rho0, const float* ux0, const float* uy0, const float* T0,
               void* stream, fftlb_handle** out);

/* Enqueue `nsteps` >= 0 explicit time steps (Sec. 3, Eq. (24) form, all derivatives by
 * windowed FFT).  The step sequence is captured once into HIP graphs and replayed. */
int fftlb_step(fftlb_handle* h, int64_t nsteps, void* stream);

/* Macroscopic fields of the current state (Eqs. (7)-(9) evaluated on f) and FP64 globals.
 * rho, ux, uy, T: device [ny][nx] float32 outputs; any of them may be NULL.
 * globals: device double[FFTLB_NGLOBALS] or NULL, receives
 *   [0] mass   = sum rho dx dy          [1] px = sum rho ux dx dy     [2] py = sum rho uy dx dy
 *   [3] energy = sum e_T dx dy with e_T = rho T - a rho^2 + K |grad rho|^2/2 + rho |u|^2/2 (Eq. (17))
 *   [4] residual = dt max_sites |sum_q v_q.grad f_q| of the last step taken (0 before any step)
 *   [5] max |u|   [6] 1 if any non-finite value was seen in the state, else 0   [7] steps taken. */
int fftlb_moments(fftlb_handle* h, float* rho, float* ux, float* uy, float* T, double* globals,
                  void* stream);

/* Copy the distribution out to / in from a device [33][ny][nx] float32 buffer. */
int fftlb_get_state(fftlb_handle* h, float* f, void* stream);
int fftlb_set_state(fftlb_handle* h, const float* f, void* stream);

/* Windowed-FFT derivative of one device [ny][nx] field g into out (may not alias g), with
 * the handle's grid and window: op 0 = D_x, 1 = D_y, 2 = D_x D_x + D_y D_y (Sec. 3.6,
 * Eq. (42) with k -> k_m; the Nyquist wavenumber of each first derivative is zero).
 * Uses the handle's stage-1 buffers: do not overlap it with fftlb_step on another stream. */
int fftlb_derivative(fftlb_handle* h, const float* g, float* out, int32_t op, void* stream);

/* Enqueue `reps` launches of one kernel of the time step, without graph capture:
 * stage 0 = convection column pass, 1 = stage-1 derivative column pass, 2 = stage-2
 * row kernel (closure of Eqs. (18)-(23)), 3 = stage-2 divergence column pass,
 * 4 = collide row kernel (Eqs. (3), (11) and the update).  Running stages 0..4 once, in
 * order, is exactly one fftlb_step; repeating a stage is for timing and leaves the
 * state meaningless until the next fftlb_set_state or fftlb_init (each stage-4 launch
 * counts as a step). */
int fftlb_run_stage(fftlb_handle* h, int32_t stage, int32_t reps, void* stream);

/* Release the handle (host memory and captured graphs); the workspace is untouched.
 * Synchronises the device first, since captured graphs may still run on caller streams. */
int fftlb_destroy(fftlb_handle* h);

/* Static string for an error code, and the thread's last detailed HIP error message. */
const char* fftlb_strerror(int code);
const char* fftlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FFTLB_H */
