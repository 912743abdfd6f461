// In-LDS Stockham FFTs for gfx950, used by every kernel of the solver.
//
// A transform of length N (a power of two) is a sequence of radix-4 passes, preceded
// by one radix-2 pass when log2 N is odd.  Each pass reads its butterfly inputs from
// LDS into registers, waits at a barrier, multiplies by the twiddles, does the
// butterfly in registers and writes the outputs back in place (Stockham autosort:
// natural order in, natural order out).
//
// Layout: element i of transform t lives at lds[t * st + i * si].  With TFAST the
// consecutive threads of a block walk consecutive transforms (column kernels, where
// transforms are interleaved with stride 1); otherwise consecutive elements of one
// transform (row kernels, where each transform is contiguous).
//
// Twiddles come from a table tw[j] = exp(-2 pi i j / N) computed in FP64 on the host.
// Direction: DIR = -1 forward (kernel exp(-i k x)), DIR = +1 inverse, both unnormalised.
#pragma once
#include <hip/hip_runtime.h>

namespace fftlb {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else {
    static_assert(R == 4, "radix");
    float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    float2 c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    // forward: y1 = b - i d, y3 = b + i d; inverse: the conjugate rotation
    float2 jd = DIR < 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, jd);
    v[3] = csub(b, jd);
  }
}

// One Stockham pass of radix R over NB transforms of length N, span P (product of the
// radices of the passes before it), executed by NTH threads.
template <int N, int R, int P, int DIR, int NTH, int NB, bool TFAST>
__device__ __forceinline__ void stockham_pass(float2* __restrict__ lds, int st, int si,
                                              const float2* __restrict__ tw, int tid) {
  constexpr int NBF = N / R;               // butterflies per transform
  constexpr int TOT = NBF * NB;            // butterflies per pass
  constexpr int BPT = (TOT + NTH - 1) / NTH;
  constexpr bool EXACT = (TOT % NTH) == 0;
  float2 v[BPT][R];
  int base[BPT], idx[BPT];
#pragma unroll
  for (int s = 0; s < BPT; ++s) {
    const int b = tid + s * NTH;
    int t, i;
    if constexpr (TFAST) {
      t = b % NB;
      i = b / NB;
    } else {
      t = b / NBF;
      i = b % NBF;
    }
    base[s] = t * st;
    idx[s] = i;
    if (EXACT || b < TOT) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[s][r] = lds[base[s] + (i + r * NBF) * si];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < BPT; ++s) {
    const int b = tid + s * NTH;
    if (EXACT || b < TOT) {
      const int i = idx[s];
      const int k = i & (P - 1);
      if constexpr (P > 1) {
        const int stride = k * (N / (P * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[r * stride];
          v[s][r] = DIR < 0 ? cmul(v[s][r], w) : cmulc(v[s][r], w);
        }
      }
      dft<R, DIR>(v[s]);
      const int j0 = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[base[s] + (j0 + r * P) * si] = v[s][r];
    }
  }
  __syncthreads();
}

template <int N, int P, int DIR, int NTH, int NB, bool TFAST>
__device__ __forceinline__ void fft_passes(float2* lds, int st, int si, const float2* __restrict__ tw,
                                           int tid) {
  if constexpr (P < N) {
    constexpr int R = (P == 1 && (ilog2(N) & 1)) ? 2 : 4;
    stockham_pass<N, R, P, DIR, NTH, NB, TFAST>(lds, st, si, tw, tid);
    fft_passes<N, P * R, DIR, NTH, NB, TFAST>(lds, st, si, tw, tid);
  }
}

// Full length-N transform of NB sequences in LDS.  Callers must have a barrier between
// their last write of the data and this call; the call ends with a barrier.
template <int N, int DIR, int NTH, int NB, bool TFAST>
__device__ __forceinline__ void fft_lds(float2* lds, int st, int si, const float2* __restrict__ tw,
                                        int tid) {
  static_assert((N & (N - 1)) == 0 && N >= 2, "power-of-two length");
  fft_passes<N, 1, DIR, NTH, NB, TFAST>(lds, st, si, tw, tid);
}

}  // namespace fftlb
