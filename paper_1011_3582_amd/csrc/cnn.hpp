// Warm-start network on gfx950: every convolution (forward, input gradient, weight gradient)
// is one implicit GEMM on the bf16 matrix cores with FP32 accumulation.
//
// A block of four waves computes a 32 x 256 block of C = A B (each wave 32 x 64: eight
// v_mfma_f32_16x16x32_bf16 per 32-deep slice of K, two row tiles sharing each B fragment).  The A tile of a slice is gathered once
// per block into LDS as bf16; B elements are gathered straight from the FP32 tensors by the
// problem's accessors and rounded to bf16 on the way into the matrix core.  Operand layouts
// of the 16x16x32 instruction (lane l of the wave):
//   A: row l % 16, k = 8 (l / 16) + i (i = 0..7)   B: k = 8 (l / 16) + i, column l % 16
//   C: row 4 (l / 16) + i (i = 0..3), column l % 16
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

typedef short s16x8 __attribute__((ext_vector_type(8)));   // bf16 bit patterns
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));  // operand type of the gfx950 bf16 MFMA
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

// Input pixel (iy, ix) feeding tap (ky, kx) of output pixel (oy, ox).
__device__ __forceinline__ void fwd_pos(const Geom& g, int ky, int kx, int oy, int ox, int& iy, int& ix) {
  if (g.kind == KIND_S1) {
    iy = wrap(oy + ky - 1, g.hin);
    ix = wrap(ox + kx - 1, g.win);
  } else if (g.kind == KIND_S2) {
    iy = wrap(2 * oy + ky - 1, g.hin);
    ix = wrap(2 * ox + kx - 1, g.win);
  } else {
    iy = wrap(oy + ky - 1, 2 * g.hin) >> 1;
    ix = wrap(ox + kx - 1, 2 * g.win) >> 1;
  }
}

// Eight consecutive K indices k .. k + 7 of one B column (n) per lane and slice: the gathers
// below compute the pixel arithmetic once for the eight (consecutive channels at one pixel, or
// consecutive pixels of one row) and fall back to element-wise gathers where the layer's sizes
// are not multiples of eight.  Elements with k >= ke or n >= N are zero.

// Forward: Z[co][p] = b[co] + sum_k W[co][k] X-gather[k][p], k = tap * cin + ci (the taps outer,
// so that eight consecutive k of a 32-channel layer are eight channels at one input pixel);
// then A = GELU(Z), or for the last layer Y = input channel + Z.
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
  __device__ float a(int m, int k, int) const { return W[(long)m * g.cin * 9 + (k % g.cin) * 9 + k / g.cin]; }
  __device__ float b(int k, int n, int z) const {
    return fwd_gather(X + z * xs, g, k % g.cin, k / g.cin, n / g.wout, n % g.wout);
  }
  __device__ void b8(int k, int n, int z, int ke, float* v) const {
    if (n >= N() || k >= ke || (g.cin & 7) || k + 8 > ke) {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (k + i < ke && n < N()) ? b(k + i, n, z) : 0.0f;
      return;
    }
    const int tap = k / g.cin, ci = k % g.cin;
    int iy, ix;
    fwd_pos(g, tap / 3, tap % 3, n / g.wout, n % g.wout, iy, ix);
    const long plane = (long)g.hin * g.win;
    const float* x = X + z * xs + ci * plane + (long)iy * g.win + ix;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = x[i * plane];
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
// dZprev[ci][p] = GELU'(Zprev[ci][p]) sum_k W^T[ci][k] dZ-gather[k][p],
// k = (tap R + r) cout + co (r over the 2 x 2 output pixels an upsampled input pixel feeds; the
// output channels inner, so that eight consecutive k are eight channels at one output pixel).
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
    const int co = k % g.cout, tap = (k / g.cout) / R();
    return W[((long)co * g.cin + m) * 9 + tap];
  }
  // Output pixel (y, x) that reads input pixel n through tap and sub-pixel q; false if none.
  __device__ bool out_pos(int tq, int n, int& y, int& x) const {
    const int r = R(), tap = tq / r, q = tq % r;
    const int ky = tap / 3, kx = tap % 3, iy = n / g.win, ix = n % g.win;
    if (g.kind == KIND_S1) {
      y = wrap(iy - ky + 1, g.hout);
      x = wrap(ix - kx + 1, g.wout);
    } else if (g.kind == KIND_S2) {
      const int ty = wrap(iy - ky + 1, g.hin), tx = wrap(ix - kx + 1, g.win);
      if ((ty | tx) & 1) return false;  // no output pixel reads this input through this tap
      y = ty >> 1;
      x = tx >> 1;
    } else {
      y = wrap(2 * iy + (q >> 1) - ky + 1, g.hout);
      x = wrap(2 * ix + (q & 1) - kx + 1, g.wout);
    }
    return true;
  }
  __device__ float b(int k, int n, int z) const {
    int y, x;
    if (!out_pos(k / g.cout, n, y, x)) return 0.0f;
    return dZ[z * zs + ((long)(k % g.cout) * g.hout + y) * g.wout + x];
  }
  __device__ void b8(int k, int n, int z, int ke, float* v) const {
    if (n >= N() || k >= ke || (g.cout & 7) || k + 8 > ke) {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (k + i < ke && n < N()) ? b(k + i, n, z) : 0.0f;
      return;
    }
    int y, x;
    if (!out_pos(k / g.cout, n, y, x)) {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.0f;
      return;
    }
    const long plane = (long)g.hout * g.wout;
    const float* d = dZ + z * zs + (k % g.cout) * plane + (long)y * g.wout + x;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = d[i * plane];
  }
  __device__ void store(int m, int n, float v, int z) const {
    const long i = z * ps + (long)m * N() + n;
    dZprev[i] = v * gelu_grad(Zprev[i]);
  }
};

// Weight gradient: dW[co][k] = sum_p dZ[co][p] X-gather[k][p] over the pixels of every
// sample; column cin * 9 gathers ones and yields db.  Blocks split the pixel sum (the
// K dimension) into chunks of every sample (z = sample * nchunks + chunk); each writes its
// partial sums to part[z][co][k], which k_wgrad_reduce adds in a fixed order (the gradient,
// and so training, is deterministic).
struct WGradProblem {
  Geom g;
  const float* X;   // layer input [n][cin][hin][win]
  const float* dZ;  // [n][cout][hout][wout]
  float* part;      // [n * nchunks][cout][cin * 9 + 1]
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
  __device__ void b8(int k, int n, int z, int ke, float* v) const {
    if (n >= N() || k >= ke || (g.wout & 7) || k + 8 > ke || n == g.cin * 9) {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (k + i < ke && n < N()) ? b(k + i, n, z) : 0.0f;
      return;
    }
    // pixels k .. k + 7 lie in one output row (k and wout are multiples of 8)
    const int ci = n / 9, tap = n % 9, ky = tap / 3, kx = tap % 3, oy = k / g.wout, ox = k % g.wout;
    const float* x = X + sample(z) * xs + (long)ci * g.hin * g.win;
    int iy, ix0;
    fwd_pos(g, ky, kx, oy, ox, iy, ix0);
    const float* row = x + (long)iy * g.win;
    if (g.kind == KIND_S1) {
      const int b0 = ox + kx - 1;  // ix of pixel i is b0 + i, wrapped
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int c = b0 + i;
        v[i] = row[c < 0 ? c + g.win : (c >= g.win ? c - g.win : c)];
      }
    } else if (g.kind == KIND_S2) {
      const int b0 = 2 * ox + kx - 1;  // ix of pixel i is b0 + 2 i, wrapped
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int c = b0 + 2 * i;
        v[i] = row[c < 0 ? c + g.win : (c >= g.win ? c - g.win : c)];
      }
    } else {
      const int b0 = ox + kx - 1, w2 = 2 * g.win;  // ix of pixel i is wrap(b0 + i, 2 win) / 2
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int c = b0 + i;
        v[i] = row[(c < 0 ? c + w2 : (c >= w2 ? c - w2 : c)) >> 1];
      }
    }
  }
  __device__ void store(int m, int n, float v, int z) const { part[((long)z * M() + m) * N() + n] = v; }
};

// dW[co][k] (k < cin * 9) and db[co] (k = cin * 9) = the sum over z = 0..nz-1 of
// part[z][co][k], accumulated in FP64 in a fixed order: a block of 256 threads takes 64
// consecutive outputs (consecutive lanes read consecutive addresses); its four thread groups
// sum the z = g, g + 4, g + 8, ... partials in order, and the four group sums are added in
// order g = 0..3.  Grid: ceil(cout * ncol / 64) blocks.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nz, int cout, int ncol,
                                                      float* __restrict__ dW, float* __restrict__ db) {
  __shared__ double grp[4][64];
  const int c = threadIdx.x & 63, gz = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + c;
  const int mn = cout * ncol;
  double acc = 0.0;
  if (i < mn)
    for (int z = gz; z < nz; z += 4) acc += part[(long)z * mn + i];
  grp[gz][c] = acc;
  __syncthreads();
  if (gz != 0 || i >= mn) return;
  const double sum = ((grp[0][c] + grp[1][c]) + grp[2][c]) + grp[3][c];
  const int m = i / ncol, k = i % ncol;
  if (k < ncol - 1)
    dW[(long)m * (ncol - 1) + k] = (float)sum;
  else
    db[m] = (float)sum;
}

// One wave: a 32 x 64 block of C (two 16-row tiles sharing each B fragment); a block of 256
// threads (four waves): 32 x 256.  Grid: x over N / 256, y over M / 32, z over the problem's
// samples (and K chunks).  Per 32-deep slice of K the block stages the 32 x 32 A tile, shared by
// its four waves, in LDS as bf16 (each element gathered once per block), then every wave gathers
// its B columns once (eight consecutive k per lane, pb.b8) and issues eight
// v_mfma_f32_16x16x32_bf16.  Every M of the network is 32 or 2, so one block row covers it.
template <class Pb>
__global__ __launch_bounds__(256) void k_gemm(Pb pb) {
  // A tile rows padded to 40 bf16 (80 bytes): the 8 values of a lane are one aligned 16-byte read
  __shared__ __attribute__((aligned(16))) short As[32][40];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 32;
  const int n0 = (blockIdx.x * 4 + wave) * 64;
  const int z = blockIdx.z;
  const int M = pb.M(), N = pb.N();
  const bool active = n0 < N;  // a wave past the end still stages A and meets the barriers
  int kb, ke;
  pb.krange(z, kb, ke);
  const int row = lane & 15, kq = (lane >> 4) * 8, crow = (lane >> 4) * 4;
  const int sr = threadIdx.x >> 3, sk = (threadIdx.x & 7) * 4;  // this thread's four staged A elements
  f32x4 acc[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[t][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + sk + e, m = m0 + sr;
      As[sr][sk + e] = bf16_bits(k < ke && m < M ? pb.a(m, k, z) : 0.0f);
    }
    __syncthreads();
    if (active) {
      const s16x8 av0 = *reinterpret_cast<const s16x8*>(&As[row][kq]);
      const s16x8 av1 = *reinterpret_cast<const s16x8*>(&As[16 + row][kq]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s16x8 bv;
        const int n = n0 + 16 * j + row;
        float bf[8];
        pb.b8(k0 + kq, n, z, ke, bf);
#pragma unroll
        for (int i = 0; i < 8; ++i) bv[i] = bf16_bits(bf[i]);
        acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av0),
                                                            __builtin_bit_cast(bf16x8, bv), acc[0][j], 0, 0, 0);
        acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av1),
                                                            __builtin_bit_cast(bf16x8, bv), acc[1][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + 16 * j + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + 16 * t + crow + i;
        if (m < M && n < N) pb.store(m, n, acc[t][j][i], z);
      }
    }
}

// Mean squared error of y against t over `count` values: dL/dy into dy, and the block
// partials of the sum of squared errors (FP64) into part[blockIdx.x] (summed by
// k_sum_partials in a fixed order).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, long count, double* part) {
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
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, long count, float v) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < count; i += (long)gridDim.x * 256) p[i] = v;
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

// ---------------------------------------------------------------------------
// Warm-start transform: prediction -> initial fields of the run.  Every sum is formed as
// per-block FP64 partials (block tree in shared memory) and one fixed-order final sum, so
// the transform is deterministic.
// ---------------------------------------------------------------------------

constexpr int kWsMaxBlocks = 1024;  // grid of the transform kernels (grid-stride loops)
constexpr int kWsSums = 4;          // partial sums per block

// Fixed-order tree sum of v over the 256 threads of a block into part[blockIdx.x * stride + c].
__device__ __forceinline__ void block_sum(double v, double* red, double* part, int stride, int c) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)blockIdx.x * stride + c] = red[0];
  __syncthreads();
}

// out[c] = sum over blocks b of part[b * stride + c], c < nval, in block order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nblocks, int stride,
                                                      int nval, double* __restrict__ out) {
  __shared__ double red[256];
  for (int c = 0; c < nval; ++c) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) acc += part[(long)b * stride + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
    __syncthreads();
  }
}

// Network input (rho0 / rho_c, T0 / T_c, T_target / T_c).
__global__ __launch_bounds__(256) void k_ws_input(const float* __restrict__ rho0, const float* __restrict__ T0,
                                                  float* __restrict__ x, long P, float irc, float itc, float tt) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256) {
    x[i] = rho0[i] * irc;
    x[P + i] = T0[i] * itc;
    x[2 * P + i] = tt;
  }
}

// Step 1: rho = clip(rho_c pred_0, rmin, rmax).
__global__ __launch_bounds__(256) void k_ws_clip(const float* __restrict__ pred, float* __restrict__ rho, long P,
                                                 float rc, float rmin, float rmax) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256)
    rho[i] = fminf(fmaxf(pred[i] * rc, rmin), rmax);
}

// Step 2: one pass of the periodic binomial filter (1 2 1)/4 along x then y, src -> dst (tmp
// holds the intermediate).  It removes the grid-scale content that upsampling layers leave in
// a prediction (the Nyquist mode exactly), which the windowed derivatives, nearly blind at
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

// Step 3a: interface weight w = |grad rho| (periodic central differences in grid units) into
// wt, and the block partials of [sum rho0, sum rho, sum w, sum T_c pred_1].
__global__ __launch_bounds__(256) void k_ws_weights(const float* __restrict__ rho0, const float* __restrict__ rho,
                                                    const float* __restrict__ pred_t, float* __restrict__ wt, int h,
                                                    int wd, float tc, double* __restrict__ part) {
  __shared__ double red[256];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < (long)h * wd; i += (long)gridDim.x * 256) {
    const int y = (int)(i / wd), x = (int)(i % wd);
    const float gx = rho[(long)y * wd + (x + 1) % wd] - rho[(long)y * wd + (x + wd - 1) % wd];
    const float gy = rho[(long)((y + 1) % h) * wd + x] - rho[(long)((y + h - 1) % h) * wd + x];
    const float g = 0.5f * sqrtf(gx * gx + gy * gy);
    wt[i] = g;
    s0 += rho0[i];
    s1 += rho[i];
    s2 += g;
    s3 += pred_t[i] * tc;
  }
  block_sum(s0, red, part, kWsSums, 0);
  block_sum(s1, red, part, kWsSums, 1);
  block_sum(s2, red, part, kWsSums, 2);
  block_sum(s3, red, part, kWsSums, 3);
}

// Step 3b: the mass deficit M0 - M (sums[0] - sums[1]) added in proportion to w (a field
// without interfaces, sum w <= 1e-6 M, is rescaled instead), clipped again; block partials
// of the new total.
__global__ __launch_bounds__(256) void k_ws_shift(float* __restrict__ rho, const float* __restrict__ wt, long P,
                                                  float rmin, float rmax, const double* __restrict__ sums,
                                                  double* __restrict__ part) {
  __shared__ double red[256];
  const bool shift = sums[2] > 1e-6 * sums[1];
  const float a = shift ? (float)((sums[0] - sums[1]) / sums[2]) : 0.0f;
  const float sc = shift ? 1.0f : (float)(sums[0] / sums[1]);
  double acc = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256) {
    const float r = fminf(fmaxf(shift ? fmaf(a, wt[i], rho[i]) : rho[i] * sc, rmin), rmax);
    rho[i] = r;
    acc += r;
  }
  block_sum(acc, red, part, kWsSums, 0);
}

// Step 3c and 4: rescale to the exact initial mass (sums[0] / sums[4]); the temperature
// uniform at the mean of the prediction (sums[3] / P), at least tmin.
__global__ __launch_bounds__(256) void k_ws_finish(float* __restrict__ rho, float* __restrict__ T, long P, float tmin,
                                                   const double* __restrict__ sums) {
  const float sc = (float)(sums[0] / sums[4]);
  const float t = fmaxf((float)(sums[3] / (double)P), tmin);
  for (long i = blockIdx.x * 256L + threadIdx.x; i < P; i += (long)gridDim.x * 256) {
    rho[i] *= sc;
    T[i] = t;
  }
}

}  // namespace cnn
}  // namespace fftlb
