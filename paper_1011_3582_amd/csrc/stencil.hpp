// The real-space stencil kernel of the flux-limiter convection scheme (see FlArgs in
// kernels.hpp).  Not a template: included by the one translation unit that launches it.
#pragma once
#include "kernels.hpp"

namespace fftlb {

// Grid: (ceil(nx / 256), ny, 32 x instances); blockIdx.z = 32 slot + (q - 1).
__global__ __launch_bounds__(256) void k_conv_fl(FlBatch B) {
  const FlArgs& A = B.c[blockIdx.z / 32];
  if (retired(B.state, A.id)) return;
  const int q = blockIdx.z % 32 + 1;  // moving population 1..32
  const int y = blockIdx.y;
  const int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= A.nx) return;
  const float vx = c_vel.vx[q], vy = c_vel.vy[q];
  const int ex = vx > 1e-3f ? 1 : vx < -1e-3f ? -1 : 0;
  const int ey = vy > 1e-3f ? 1 : vy < -1e-3f ? -1 : 0;
  const float a_i = (ex != 0 && ey != 0) ? 1.41421356237309505f : 1.0f;
  const float speed = sqrtf(c_vel.v2[q]);
  const float c = speed * A.cf / a_i;
  const int nx = A.nx, ny = A.ny;
  const float* g = A.f + (long)q * nx * ny;
  // node J + n e, periodic (|n| <= 2 < nx, ny)
  auto at = [&](int n) {
    const int xx = (x + n * ex + 2 * nx) % nx, yy = (y + n * ey + 2 * ny) % ny;
    return g[(long)yy * nx + xx];
  };
  const float f0 = at(0), fp1 = at(1), fm1 = at(-1), fm2 = at(-2);
  const float fp = f0 + 0.5f * (1.0f - c) * mcd_limited(f0 - fm1, fp1 - f0);
  const float fm = fm1 + 0.5f * (1.0f - c) * mcd_limited(fm1 - fm2, f0 - fm1);
  A.out[(long)(q - 1) * nx * ny + (long)y * nx + x] = speed * A.rdr / (a_i * nx) * (fp - fm);
}

}  // namespace fftlb
