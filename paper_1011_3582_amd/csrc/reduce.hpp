// Global reductions and the batch poll; included by the API translation unit only.
#pragma once
#include "launch.hpp"

namespace fftlb {

// Sum the per-block partials in FP64, in a fixed order, into the 8 globals.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part_d, int nd,
                                                  const float* __restrict__ part_f, int nf,
                                                  double cell, double dt, double steps,
                                                  double* __restrict__ out) {
  __shared__ double sd[256][4];
  __shared__ float sf[256][4];
  const int tid = threadIdx.x;
  double s[4] = {0, 0, 0, 0};
  float um = 0.0f, bd = 0.0f, rr = 0.0f;
  for (int i = tid; i < nd; i += 256) {
    for (int c = 0; c < 4; ++c) s[c] += part_d[6 * i + c];
    um = fmaxf(um, (float)part_d[6 * i + 4]);
    bd = fmaxf(bd, (float)part_d[6 * i + 5]);
  }
  for (int i = tid; i < nf; i += 256) {
    rr = fmaxf(rr, part_f[2 * i]);
    bd = fmaxf(bd, part_f[2 * i + 1]);
  }
  for (int c = 0; c < 4; ++c) sd[tid][c] = s[c];
  sf[tid][0] = um;
  sf[tid][1] = bd;
  sf[tid][2] = rr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      for (int c = 0; c < 4; ++c) sd[tid][c] += sd[tid + w][c];
      for (int c = 0; c < 3; ++c) sf[tid][c] = fmaxf(sf[tid][c], sf[tid + w][c]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = sd[0][0] * cell;
    out[1] = sd[0][1] * cell;
    out[2] = sd[0][2] * cell;
    out[3] = sd[0][3] * cell;
    out[4] = (double)sf[0][2] * dt;
    out[5] = sf[0][0];
    out[6] = sf[0][1] > 0.0f ? 1.0 : 0.0;
    out[7] = steps;
  }
}

// Uniform temperature shift dT = (energy - E) / M from the globals g (g[3] = E, g[0] = M) of
// the state: T += dT at every site of the temperature plane.
__global__ __launch_bounds__(256) void k_shift_temperature(float* __restrict__ T, long P,
                                                           const double* __restrict__ g, double energy) {
  const double dT = (energy - g[3]) / g[0];
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256)
    T[i] = (float)((double)T[i] + dT);
}

// Per-instance convergence bookkeeping of a batch, in device memory.
struct BatchState {
  int* state;              // 0 running, 1 converged, 2 non-finite
  int* below;              // consecutive polls with residual < tol
  long long* steps;        // steps taken
  long long* first_below;  // steps at the first poll of the current run below tol (-1: none)
  double* residual;        // dt max |sum_q v_q.grad f_q| of the last step
};

// Where the poll finds an instance's collide partials.
struct PollInfo {
  const float* part_f;  // [nblk][2] max |D.(rho u)|, non-finite flag
  int nblk;
  float dt;
};

// One block per instance, after `nsteps` steps of every running instance and the residual
// pass: the residual (the same quantity as global [4]), and retirement
// once it has stayed below `tol` for `consecutive` polls, or at once on a non-finite value.
__global__ __launch_bounds__(256) void k_batch_poll(const PollInfo* __restrict__ info, BatchState b, int nsteps,
                                                    double tol, int consecutive) {
  const int i = blockIdx.x;
  if (b.state[i]) return;
  const PollInfo In = info[i];
  const int tid = threadIdx.x;
  float r = 0.0f, bad = 0.0f;
  for (int k = tid; k < In.nblk; k += 256) {
    r = fmaxf(r, In.part_f[2 * k]);
    bad = fmaxf(bad, In.part_f[2 * k + 1]);
  }
  __shared__ float red[4][2];
  r = wave_max(r);
  bad = wave_max(bad);
  if (tid % 64 == 0) {
    red[tid / 64][0] = r;
    red[tid / 64][1] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) {
      r = fmaxf(r, red[w][0]);
      bad = fmaxf(bad, red[w][1]);
    }
    const long long steps = b.steps[i] + nsteps;
    b.steps[i] = steps;
    const double res = (double)r * (double)In.dt;
    b.residual[i] = res;
    if (bad > 0.0f || !(res <= 1e300)) {
      b.state[i] = 2;
    } else if (res < tol) {
      if (b.below[i] == 0) b.first_below[i] = steps;
      if (++b.below[i] >= consecutive) b.state[i] = 1;
    } else {
      b.below[i] = 0;
      b.first_below[i] = -1;
    }
  }
}

}  // namespace fftlb
