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
 *    enqueued on it asynchronously.  Calls that wait are said so below: fftlb_init (it
 *    uploads small tables and captures the step graphs), fftlb_poll, fftlb_set_plan (for
 *    the handle's last graph replay), fftlb_autotune, fftlb_destroy and the batch calls.
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
#define FFTLB_EUNSTABLE (-4) /* non-finite values in the state (fftlb_poll, fftlb_batch_run) */

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
 *  filter_order  0 = exact wavenumber k, 1..4 = windowed k_1..k_4 (Eqs. (44)-(47)), 5 = the
 *                second-order central difference of Sec. 3.1 for every derivative (the CD + CD
 *                comparison scheme): on the periodic grid the stencil (g[J+1] - g[J-1]) / (2 d)
 *                is the multiplier i sin(k d) / d, applied in the same spectral passes.  6 = the
 *                nine-point stencils of the NPS scheme (Sec. 3.1; B = 1/12 for the first
 *                derivatives, F = 1/6 for the Laplacian of the pressure tensor; second
 *                derivatives of theta are compositions of first ones) for every derivative of the
 *                force, and with convection 0 for the convection term too; dx must equal dy.
 *                The stencils couple the axes, so every derivative goes through column passes
 *                (5 more spectral planes of workspace, and a step of five kernels).
 *  precision     storage of the distribution: 0 = FP32; 1 = compensated, f = hi + lo with
 *                both parts FP32 (|lo| at most half an ulp of hi): each update adds its
 *                increment exactly, so increments below half an FP32 ulp of f, which an
 *                FP32 state loses, still accumulate (long relaxations to small residuals);
 *                33 more planes of workspace and of collide traffic.  Arithmetic is FP32
 *                in both (the transforms and the convection term take hi).
 *  convection    scheme of the convection term v.grad f: 0 = the derivative operator of
 *                filter_order (windowed FFT, or CD with filter_order 5); 1 = Lax-Wendroff
 *                (Sec. 3.1, Eq. (ML-)); 2 = MLW1, LW plus the dispersion correction R3 (Eq. (R3));
 *                3 = MLW2, LW plus R3 and the dissipation correction R4 (Eq. (R4=)); 4 = the flux
 *                limiter with the MCD limiter along each population's characteristic line (Sec. 3.1,
 *                Eq. (FL); dx must equal dy), computed in real space and taken to spectra by row
 *                transforms (32 more planes of workspace).  For 1..3 the
 *                one-dimensional stencils act along x and along y and their updates add; the
 *                CFL numbers are c = v_x dt/dx and v_y dt/dy.  On the periodic grid every such
 *                stencil is a multiplication of the spectrum, applied in a column pass over all
 *                32 moving populations (a step then runs five kernels instead of four).  With
 *                filter_order 5 these are the paper's LW + CD, MLW1 + CD and MLW2 + CD schemes. */
typedef struct fftlb_config {
  int32_t nx, ny;
  double dx, dy, dt;
  double tau, K, H, zeta, q;
  double a, b;
  int32_t filter_order;
  int32_t precision;
  int32_t convection;
} fftlb_config;

typedef struct fftlb_handle fftlb_handle;

/* Bytes of device workspace fftlb_init needs for `cfg` (about 88 * nx * ny * 4 bytes; 121 for
 * a compensated state).
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
 * windowed FFT).  The step sequence is captured into HIP graphs of 1, 2, 4, 8 and 16
 * steps by fftlb_init (and again after a plan change) and replayed: floor(nsteps / 16)
 * replays of the 16-step graph and one of each graph in the binary digits of the rest. */
int fftlb_step(fftlb_handle* h, int64_t nsteps, void* stream);

/* Macroscopic fields of the current state (Eqs. (7)-(9) evaluated on f) and FP64 globals.
 * rho, ux, uy, T: device [ny][nx] float32 outputs; any of them may be NULL.
 * globals: device double[FFTLB_NGLOBALS] or NULL, receives
 *   [0] mass   = sum rho dx dy          [1] px = sum rho ux dx dy     [2] py = sum rho uy dx dy
 *   [3] energy = sum e_T dx dy with e_T = rho T - a rho^2 + K |grad rho|^2/2 + rho |u|^2/2 (Eq. (17))
 *   [4] residual = dt max_sites |D.(rho u)| of the current state, D the windowed derivative:
 *       in exact arithmetic the sum over populations of the convection terms of the next
 *       step, i.e. max |rho^{n+1} - rho^n| (the collision and the force conserve mass)
 *   [5] max |u|   [6] 1 if any non-finite value was seen in the state, else 0   [7] steps taken. */
int fftlb_moments(fftlb_handle* h, float* rho, float* ux, float* uy, float* T, double* globals,
                  void* stream);

/* Synchronising check of the current state: the FP64 globals of fftlb_moments, computed on
 * `stream` into the workspace and copied to `globals` (HOST double[FFTLB_NGLOBALS], or
 * NULL); waits for `stream`.  Returns FFTLB_EUNSTABLE when the non-finite flag (global [6])
 * is set, i.e. some rho, u, T or force coefficient of the state is NaN or infinite
 * (a blown-up run), else FFTLB_OK; the globals are written in both cases. */
int fftlb_poll(fftlb_handle* h, double* globals, void* stream);

/* Match the total energy: shift the temperature field of the current state uniformly by
 * dT = (energy - E) / M, with E and M the FP64 total energy (Eq. (17), as global [3] of
 * fftlb_moments) and mass (global [0]) of the current state, and restart from the local
 * equilibrium f := f^eq(rho, u, T + dT) of Eq. (3).  Since T enters e_T only through rho T,
 * the new state has total energy `energy` (up to FP32 rounding of T + dT).  For starting a
 * run from predicted fields with the invariants of a given initial state: the mass through
 * the fields themselves, the energy through this call.  Asynchronous on `stream`; a
 * non-positive T + dT is the caller's responsibility (check with fftlb_poll). */
int fftlb_match_energy(fftlb_handle* h, double energy, void* stream);

/* Copy the distribution out to / in from a device [33][ny][nx] float32 buffer.  For a
 * compensated state get_state copies hi (f rounded to FP32) and set_state sets lo to 0. */
int fftlb_get_state(fftlb_handle* h, float* f, void* stream);
int fftlb_set_state(fftlb_handle* h, const float* f, void* stream);

/* Windowed-FFT derivative of one device [ny][nx] field g into out (may not alias g), with
 * the handle's grid and window: op 0 = D_x, 1 = D_y, 2 = D_x D_x + D_y D_y (Sec. 3.6,
 * Eq. (42) with k -> k_m; the Nyquist wavenumber of each first derivative is zero).  With
 * filter_order 6 these are the NPS stencils' D_x, D_y and nine-point Laplacian (Sec. 3.1).
 * Uses the handle's stage-1 buffers: do not overlap it with fftlb_step on another stream. */
int fftlb_derivative(fftlb_handle* h, const float* g, float* out, int32_t op, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): fftlb_derivative without a handle or workspace.  The
 * windowed derivative op (0 = D_x, 1 = D_y, 2 = D_x D_x + D_y D_y) of the device [ny][nx]
 * field g into out (may not alias g), for the grid, spacings and window of `cfg` (its other
 * fields are checked but unused); results equal fftlb_derivative's up to FP32 rounding of
 * the tables (computed here on the device).  The two spectral planes and the tables live in
 * a static device array the library holds on each GPU it runs on until the process ends
 * (about 2.1 MB): nx * ny may not exceed 512 * 512 (FFTLB_EINVAL, with the reason in
 * fftlb_last_error); filter_order 6 (the NPS stencils) is not available here (FFTLB_EINVAL).
 * It calls no allocating routine.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller; calls on one stream are ordered. */
int fftlb_derivative_static(const fftlb_config* cfg, const float* g, float* out, int32_t op, void* stream);

/* Enqueue `reps` launches of one kernel of the time step, without graph capture:
 * stage 0 = stage-1 derivative column pass together with the column pass that forms the
 * y-parts v_y D_y f of the convection terms of 16 of the 24 populations with v_y != 0 from f
 * (one launch), 1 = stage-2 row kernel (closure of Eqs. (18)-(23)), 2 = stage-2 divergence
 * column pass together with the y-parts of the other 8, 3 = collide row kernel (the x-parts
 * v_x D_x f from f^n, Eqs. (3), (11) and the update).  Running stages
 * 0..3 once, in order, is exactly one fftlb_step; repeating a stage is for timing and
 * leaves the state meaningless until the next fftlb_set_state or fftlb_init (each
 * stage-3 launch counts as a step).  With a finite-difference convection scheme or the NPS
 * stencils (fftlb_config.convection != 0 or filter_order 6) stage 0 is the stage-1 derivative
 * pass followed by the scheme's convection pass (two launches; with the flux limiter the
 * stencil kernel and the row transforms of its 32 planes) and stage 2 the divergence pass
 * alone.  Other stage numbers: FFTLB_EINVAL. */
int fftlb_run_stage(fftlb_handle* h, int32_t stage, int32_t reps, void* stream);

/* Column-pass plan of a handle: complex columns per block of the convection pass (pairs of
 * real columns of f, or spectral columns with a finite-difference scheme) and of the
 * derivative passes (powers of two up to 16, at most the tile width min(16, the
 * largest power of two dividing nx/2), and within 64 KB of LDS: ny * conv_cols <= 8192,
 * 3 * ny * multi_cols <= 8192), and the largest radix of the column transforms of each
 * (8 or 16).  In the step both derivative passes run inside convection launches, with
 * their radix and block size and conv_cols / 3 columns per block (rounded down to a
 * power of two, at least 1); multi_cols and multi_radix set the derivative passes of the
 * diagnostics (fftlb_moments, the batch residual) and of fftlb_derivative.  fftlb_init picks
 * the widest tiles and radix 16.  fftlb_set_plan waits for the last replay of the handle's
 * step graphs (they may still be queued on the caller's stream), destroys them and captures
 * the new plan's graphs; the new plan applies to everything enqueued after the call.
 * Plans change speed only: the results of any two plans agree to FP32 rounding of the
 * column transforms. */
typedef struct fftlb_plan {
  int32_t conv_cols, multi_cols, conv_radix, multi_radix;
} fftlb_plan;
int fftlb_get_plan(const fftlb_handle* h, fftlb_plan* plan);
int fftlb_set_plan(fftlb_handle* h, const fftlb_plan* plan);

/* Autotuner: time every column plan of the handle's grid size (`reps` launches each, on
 * `stream`, synchronising) on the handle's current state and set the fastest.  The state
 * is restored afterwards (everything derived from f is recomputed from it), so the trajectory is
 * unchanged.  With `cache_path` (a text file, NULL for none) a plan already stored there
 * for this device architecture and grid size is used without timing, and a newly timed
 * plan is appended.  *best (may be NULL) receives the plan. */
int fftlb_autotune(fftlb_handle* h, int32_t reps, const char* cache_path, void* stream, fftlb_plan* best);

/* Release the handle (host memory and captured graphs); the workspace is untouched.
 * Synchronises the device first, since captured graphs may still run on caller streams. */
int fftlb_destroy(fftlb_handle* h);

/* ------------------------------------------------------------------------------------
 * Batches: up to FFTLB_MAX_BATCH independent instances, of any mix of supported grid
 * sizes and parameters, advanced together.  Each launch of a step kernel covers every
 * running instance of one grid size; fftlb_batch_run replays one captured HIP graph of
 * `poll_every` steps of all running instances followed by an on-device poll that retires
 * converged instances (their blocks exit at once in later launches), so the host only
 * reads the retirement flags between replays.  The residual is global [4] of
 * fftlb_moments, dt max_sites |D.(rho u)| = max |rho^{n+1} - rho^n| in exact arithmetic,
 * formed from the momentum field so that its FP32 floor is set by the rounding of rho u
 * (far below 1e-8 at the paper's dt), not by differences of stored densities or by the
 * rounding of the 32 convection terms whose sum it is.
 * ------------------------------------------------------------------------------------ */
#define FFTLB_MAX_BATCH 1024
typedef struct fftlb_batch fftlb_batch;

/* Device workspace for a batch of n configurations (the sum of the instances'
 * workspaces plus bookkeeping). */
int fftlb_batch_workspace_bytes(int32_t n, const fftlb_config* cfgs, size_t* bytes);

/* Initialise n instances on `workspace` as fftlb_init does for each; rho0[i] .. T0[i] are
 * host arrays of n device pointers to instance i's [ny][nx] initial fields (read during
 * the call only).  Synchronises `stream`. */
int fftlb_batch_create(int32_t n, const fftlb_config* cfgs, void* workspace, size_t ws_bytes,
                       const float* const* rho0, const float* const* ux0, const float* const* uy0,
                       const float* const* T0, void* stream, fftlb_batch** out);

/* fftlb_autotune for each grid size of the batch (on its first instance), applied to
 * every instance of that size. */
int fftlb_batch_autotune(fftlb_batch* b, int32_t reps, const char* cache_path, void* stream);

/* Advance every running instance until all have retired or at least `max_steps` more
 * steps were taken (a multiple of poll_every, 1..1000).  An instance retires as
 * converged (state 1) when its residual is below `tol` at `consecutive` successive polls,
 * or as unstable (state 2) at a non-finite value.  Synchronises `stream`.  Returns
 * FFTLB_EUNSTABLE when some instance is in state 2 at the end of the call (the others were
 * advanced as usual; fftlb_batch_status tells which), else FFTLB_OK. */
int fftlb_batch_run(fftlb_batch* b, double tol, int32_t consecutive, int32_t poll_every, int64_t max_steps,
                    void* stream);

/* Host arrays of n entries (each may be NULL): steps taken, steps at the first of the
 * `consecutive` polls below tol (-1 unless converged), last polled residual, state
 * (0 running, 1 converged, 2 non-finite).  Synchronises the device. */
int fftlb_batch_status(fftlb_batch* b, int64_t* steps, int64_t* steps_to_tol, double* residual, int32_t* state);

/* The handle of instance i (owned by the batch: fftlb_moments, fftlb_get_state, ... work
 * on it; do not destroy it). */
int fftlb_batch_instance(fftlb_batch* b, int32_t i, fftlb_handle** h);

/* Release the batch and its instance handles; the workspace is untouched. */
int fftlb_batch_destroy(fftlb_batch* b);

/* Static string for an error code, and the thread's last detailed HIP error message. */
const char* fftlb_strerror(int code);
const char* fftlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FFTLB_H */
