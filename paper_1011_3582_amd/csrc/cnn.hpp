// Warm-start network on gfx950: every convolution (forward, input gradient, weight gradient)
// is one implicit GEMM on the bf16 matrix cores with FP32 accumulation.
//
// A wave computes a 16 x 64 block of C = A B (four v_mfma_f32_16x16x16_bf16 per 16-deep
// slice of K); A and B elements are gathered straight from the FP32 tensors in global
// memory by the problem's accessors and rounded to bf16 on the way into the matrix core.
// Operand layouts of the 16x16x16 instruction (lane l of the wave, i = 0..3):
//   A: row l % 16, k = 4 (l / 16) + i      B: k = 4 (l / 16) + i, column l % 16
//   C: row 4 (l / 16) + i, column l % 16
//
// Network (3 x 3 taps, periodic padding, cross-correlation; per layer W[Cout][Cin][3][3], b):
//   1: 3 -> 32 conv   2: 32 -> 32 conv stride 2   3: 32 -> 32 conv stride 2
//   4: up x2, 32 -> 32 conv   5: up x2, 32 -> 32 conv   6: 32 -> 2 conv, linear
// GELU (erf form) after layers 1-5; output = input channels 0, 1 + layer-6 output.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fftlb {
namespace cnn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 6;
constexpr int kCin[kLayers] = {3, 32, 32, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 32, 32, 2};
enum : int { KIND_S1 = 0, KIND_S2 = 1, KIND_UP = 2 };
constexpr int kKind[kLayers] = {KIND_S1, KIND_S2, KIND_S2, KIND_UP, KIND_UP, KIND_S1};

// Parameter offsets in the flat vector: W then b per layer.
constexpr int param_offset(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += kCout[i] * kCin[i] * 9 + kCout[i];
  return o;
}
constexpr int kParams = param_offset(kLayers);

// bf16 bits of x, rounded to nearest even (finite inputs).
__device__ __forceinline__ short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct Geom {
  int cin, cout, hin, win, hout, wout, kind;
};

// Input value feeding tap `tap` (ky = tap / 3, kx = tap % 3) of output pixel (oy, ox).
__device__ __forceinline__ float fwd_gather(const float* __restrict__ X, const Geom& g, int ci, int tap, int oy,
                                            int ox) {
  const int ky = tap / 3, kx = tap % 3;
  int iy, ix;
  if (g.kind == KIND_S1) {
    iy = wrap(oy + ky - 1, g.hin);
    ix = wrap(ox + kx - 1, g.win);
  } else if (g.kind == KIND_S2) {
    iy = wrap(2 * oy + ky - 1, g.hin);
    ix = wrap(2 * ox + kx - 1, g.win);
  } else {  // nearest upsampling by 2, then the stride-1 tap
    iy = wrap(oy + ky - 1, 2 * g.hin) >> 1;
    ix = wrap(ox + kx - 1, 2 * g.win) >> 1;
  }
  return X[((long)ci * g.hin + iy) * g.win + ix];
}

// Forward: Z[co][p] = b[co] + sum_k W[co][k] X-gather[k][p], k = (ci, tap); then
// A = GELU(Z), or for the last layer Y = input channel + Z.
struct FwdProblem {
  Geom g;
  const float* X;      // [n][cin][hin][win]
  const float* W;      // [cout][cin * 9]
  const float* bias;   // [cout]
  float* Z;            // [n][cout][hout][wout]
  float* A;            // GELU(Z) or null
  const float* resid;  // network input [n][3][hout][wout] (last layer) or null
  float* Y;            // [n][2][hout][wout] (last layer) or null
  long xs, zs, rs;     // per-sample strides of X, Z (and A, Y), resid
  __device__ int M() const { return g.cout; }
  __device__ int N() const { return g.hout * g.wout; }
  __device__ void krange(int, int& b, int& e) const {
    b = 0;
    e = g.cin * 9;
  }
  __device__ int sample(int z) const { return z; }
  __device__ float a(int m, int k, int) const { return W[(long)m * g.cin * 9 + k]; }
  __device__ float b(int k, int n, int z) const {
    return fwd_gather(X + z * xs, g, k / 9, k % 9, n / g.wout, n % g.wout);
  }
  __device__ void store(int m, int n, float v, int z) const {
    const long i = z * zs + (long)m * N() + n;
    const float zz = v + bias[m];
    Z[i] = zz;
    if (A) A[i] = gelu(zz);
    if (Y) Y[i] = resid[z * rs + (long)m * N() + n] + zz;
  }
};

// Input gradient of a layer whose input is the GELU output of the layer before:
// dZprev[ci][p] = GELU'(Zprev[ci][p]) sum_k W^T[ci][k] dZ-gather[k][p], k = (co, tap, r),
// r over the 2 x 2 output pixels an upsampled input pixel feeds.
struct BwdDataProblem {
  Geom g;
  const float* W;      // [cout][cin][9]
  const float* dZ;     // [n][cout][hout][wout]
  const float* Zprev;  // [n][cin][hin][win]
  float* dZprev;       // [n][cin][hin][win]
  long zs, ps;         // per-sample strides of dZ and Zprev / dZprev
  __device__ int R() const { return g.kind == KIND_UP ? 4 : 1; }
  __device__ int M() const { return g.cin; }
  __device__ int N() const { return g.hin * g.win; }
  __device__ void krange(int, int& b, int& e) const {
    b = 0;
    e = g.cout * 9 * R();
  }
  __device__ int sample(int z) const { return z; }
  __device__ float a(int m, int k, int) const {
    const int r = R(), co = k / (9 * r), tap = (k / r) % 9;
    return W[((long)co * g.cin + m) * 9 + tap];
  }
  __device__ float b(int k, int n, int z) const {
    const int r = R(), co = k / (9 * r), tap = (k / r) % 9, q = k % r;
    const int ky = tap / 3, kx = tap % 3, iy = n / g.win, ix = n % g.win;
    int y, x;
    if (g.kind == KIND_S1) {
      y = wrap(iy - ky + 1, g.hout);
      x = wrap(ix - kx + 1, g.wout);
    } else if (g.kind == KIND_S2) {
      const int ty = wrap(iy - ky + 1, g.hin), tx = wrap(ix - kx + 1, g.win);
      if ((ty | tx) & 1) return 0.0f;  // no output pixel reads this input through this tap
      y = ty >> 1;
      x = tx >> 1;
    } else {
      y = wrap(2 * iy + (q >> 1) - ky + 1, g.hout);
      x = wrap(2 * ix + (q & 1) - kx + 1, g.wout);
    }
    return dZ[z * zs + ((long)co * g.hout + y) * g.wout + x];
  }
  __device__ void store(int m, int n, float v, int z) const {
    const long i = z * ps + (long)m * N() + n;
    dZprev[i] = v * gelu_grad(Zprev[i]);
  }
};

// Weight gradient: dW[co][k] = sum_p dZ[co][p] X-gather[k][p] over the pixels of every
// sample; column cin * 9 gathers ones and yields db.  Blocks split the pixel sum (the
// K dimension) into chunks and accumulate with atomic adds.
struct WGradProblem {
  Geom g;
  const float* X;   // layer input [n][cin][hin][win]
  const float* dZ;  // [n][cout][hout][wout]
  float* dW;        // [cout][cin * 9]
  float* db;        // [cout]
  long xs, zs;
  int chunk, nchunks;
  __device__ int M() const { return g.cout; }
  __device__ int N() const { return g.cin * 9 + 1; }
  __device__ void krange(int z, int& b, int& e) const {
    const int c = z % nchunks, P = g.hout * g.wout;
    b = c * chunk;
    e = b + chunk < P ? b + chunk : P;
  }
  __device__ int sample(int z) const { return z / nchunks; }
  __device__ float a(int m, int k, int z) const { return dZ[sample(z) * zs + (long)m * g.hout * g.wout + k]; }
  __device__ float b(int k, int n, int z) const {
    if (n == g.cin * 9) return 1.0f;
    return fwd_gather(X + sample(z) * xs, g, n / 9, n % 9, k / g.wout, k % g.wout);
  }
  __device__ void store(int m, int n, float v, int) const {
    if (n < g.cin * 9)
      atomicAdd(&dW[(long)m * g.cin * 9 + n], v);
    else
      atomicAdd(&db[m], v);
  }
};

// One wave: a 16 x 64 block of C; a block of 256 threads: 16 x 256.  Grid: x over N / 256,
// y over M / 16, z over the problem's samples (and K chunks).
template <class Pb>
__global__ __launch_bounds__(256) void k_gemm(Pb pb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 16;
  const int n0 = (blockIdx.x * 4 + wave) * 64;
  const int z = blockIdx.z;
  const int M = pb.M(), N = pb.N();
  if (n0 >= N) return;  // whole wave past the end (no barriers in this kernel)
  int kb, ke;
  pb.krange(z, kb, ke);
  const int row = lane & 15, kq = (lane >> 4) * 4;
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x4 av;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + kq + i, m = m0 + row;
      av[i] = bf16_bits(k < ke && m < M ? pb.a(m, k, z) : 0.0f);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf16x4 bv;
      const int n = n0 + 16 * j + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + kq + i;
        bv[i] = bf16_bits(k < ke && n < N ? pb.b(k, n, z) : 0.0f);
      }
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + 16 * j + row;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + kq + i;
      if (m < M && n < N) pb.store(m, n, acc[j][i], z);
    }
  }
}

// Mean squared error of y against t over `count` values: dL/dy into dy, the sum of squared
// errors added to *sse (FP64).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, long count, double* sse) {
  __shared__ double red[256];
  double acc = 0.0;
  const float s = 2.0f / (float)count;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
    const float d = y[i] - t[i];
    dy[i] = s * d;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(sse, red[0]);
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, long count, float v) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < count; i += (long)gridDim.x * 256) p[i] = v;
}

__global__ void k_fill_d(double* p, int count) {
  if ((int)threadIdx.x < count) p[threadIdx.x] = 0.0;
}

// Adam with bias correction (bc1 = 1 - beta1^t, bc2 = 1 - beta2^t).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int count, float lr,
                                              float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Warm start: network input (rho0 / rho_c, T0 / T_c, T_target / T_c) and the FP64 sum of rho0.
__global__ __launch_bounds__(256) void k_ws_input(const float* __restrict__ rho0, const float* __restrict__ T0,
                                                  float* __restrict__ x, long P, float irc, float itc, float tt,
                                                  double* sum) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256) {
    x[i] = rho0[i] * irc;
    x[P + i] = T0[i] * itc;
    x[2 * P + i] = tt;
    acc += rho0[i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(sum, red[0]);
}

// Network output -> density clamped to the physical range; FP64 sums of the density
// (sums[1]) and of the predicted temperature (sums[2]).
__global__ __launch_bounds__(256) void k_ws_output(const float* __restrict__ y, float* __restrict__ rho, long P,
                                                   float rc, float tc, float rmin, float rmax, double* sums) {
  __shared__ double red[256][2];
  double acc = 0.0, acct = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256) {
    const float r = fminf(fmaxf(y[i] * rc, rmin), rmax);
    rho[i] = r;
    acc += r;
    acct += y[P + i] * tc;
  }
  red[threadIdx.x][0] = acc;
  red[threadIdx.x][1] = acct;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x][0] += red[threadIdx.x + w][0];
      red[threadIdx.x][1] += red[threadIdx.x + w][1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&sums[1], red[0][0]);
    atomicAdd(&sums[2], red[0][1]);
  }
}

// One pass of the periodic binomial filter (1 2 1)/4 along x then y, src -> dst (tmp holds
// the intermediate).  It removes the grid-scale content that upsampling layers leave in a
// prediction (the Nyquist mode exactly), which the windowed derivatives, nearly blind at
// those wavenumbers, would otherwise carry for a long time; it conserves the total.
__global__ __launch_bounds__(256) void k_ws_smooth_x(const float* __restrict__ src, float* __restrict__ tmp, int h,
                                                     int w) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < (long)h * w; i += (long)gridDim.x * 256) {
    const int y = (int)(i / w), x = (int)(i % w);
    const long r = (long)y * w;
    tmp[i] = 0.25f * src[r + (x + w - 1) % w] + 0.5f * src[i] + 0.25f * src[r + (x + 1) % w];
  }
}

__global__ __launch_bounds__(256) void k_ws_smooth_y(const float* __restrict__ tmp, float* __restrict__ dst, int h,
                                                     int w) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < (long)h * w; i += (long)gridDim.x * 256) {
    const int y = (int)(i / w), x = (int)(i % w);
    dst[i] = 0.25f * tmp[(long)((y + h - 1) % h) * w + x] + 0.5f * tmp[i] + 0.25f * tmp[(long)((y + 1) % h) * w + x];
  }
}

// Interface weight w = |grad rho| (central differences, periodic) into w, and its FP64
// total into sums[3].
__global__ __launch_bounds__(256) void k_ws_interface(const float* __restrict__ rho, float* __restrict__ w, int h,
                                                      int wd, double* sums) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < (long)h * wd; i += (long)gridDim.x * 256) {
    const int y = (int)(i / wd), x = (int)(i % wd);
    const float gx = rho[(long)y * wd + (x + 1) % wd] - rho[(long)y * wd + (x + wd - 1) % wd];
    const float gy = rho[(long)((y + 1) % h) * wd + x] - rho[(long)((y + h - 1) % h) * wd + x];
    const float g = 0.5f * sqrtf(gx * gx + gy * gy);
    w[i] = g;
    acc += g;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&sums[3], red[0]);
}

// Restore the initial total mass M0 = sums[0] from the prediction's sums[1] by adding
// (M0 - M) w / sum(w): the mass goes to or comes from the interfaces, which move slightly,
// while the bulk densities stay at the predicted values (a uniform rescaling would move
// both phases off coexistence, and that relaxes only by slow evaporation and
// condensation).  Without interfaces (sum(w) == 0) the density is rescaled.  The
// temperature is the mean of the prediction, uniform (the model's equilibria are
// isothermal, and a non-uniform start would relax only by slow conduction).
__global__ __launch_bounds__(256) void k_ws_project(float* __restrict__ rho, const float* __restrict__ w,
                                                    float* __restrict__ T, long P, float tmin, const double* sums) {
  const double dm = sums[0] - sums[1];
  const bool shift = sums[3] > 1e-6 * sums[1];
  const float a = shift ? (float)(dm / sums[3]) : 0.0f;
  const float sc = shift ? 1.0f : (float)(sums[0] / sums[1]);
  const float t = fmaxf((float)(sums[2] / (double)P), tmin);
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256) {
    rho[i] = shift ? rho[i] + a * w[i] : rho[i] * sc;
    T[i] = t;
  }
}

}  // namespace cnn
}  // namespace fftlb
