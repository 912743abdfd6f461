// In-LDS Stockham FFTs for gfx950, used by every kernel of the solver.
//
// A transform of length N = 2^p or 3 * 2^p is a sequence of radix-16 (or radix-8) passes,
// preceded by a radix-3 pass when 3 divides N and by one smaller power-of-two pass when
// log2 of the power-of-two part is not a multiple of 4 (or 3).  Each pass reads
// its butterfly inputs from LDS into registers, waits at a barrier, multiplies by the
// twiddles, does the butterfly in registers and writes the outputs back in place
// (Stockham autosort: natural order in, natural order out).  With radix 16 a 1024-point
// transform takes three passes, and a thread holds 16 complex values per pass.
//
// Layout: element i of transform t lives at lds[pad(off + t * st + i * SI)], where pad()
// inserts one empty slot after every 32 elements so that the strided accesses of the
// passes spread over the LDS banks.  When the caller's layout keeps off + t * st a
// multiple of 32 (ALIGNED), the 2R accesses of a butterfly are one runtime base address
// plus compile-time offsets, which the hardware takes as immediate offsets: the address
// arithmetic does not grow with the radix.  With TFAST the consecutive threads of a block
// walk consecutive transforms (column kernels, transforms interleaved with stride SI);
// otherwise consecutive butterflies of one transform (row kernels, contiguous transforms).
//
// Twiddles come from a table tw[j] = exp(-2 pi i j / N) computed in FP64 on the host; the
// kernels rearrange it into per-pass tables in LDS first (TWL, see build_twiddles), so
// that every power is one conflict-free LDS read.
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
constexpr bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
// Transform lengths handled here: 2^p, or 3 * 2^p (one radix-3 pass first).
constexpr bool fft_length_ok(int n) { return n >= 2 && (is_pow2(n) || (n % 3 == 0 && is_pow2(n / 3))); }

// Padded LDS element index (see the file comment) and the padded size of n elements.
__host__ __device__ constexpr int pad(int e) { return e + (e >> 5); }
__host__ __device__ constexpr int padded_size(int n) { return n + (n >> 5) + 1; }

// Returns v unchanged but opaque to the optimiser.  Index arithmetic derived from the
// result is recomputed where it is used instead of being hoisted out of loops and kept
// live (the many per-pass LDS addresses would otherwise exhaust the VGPRs).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Thread index below NT, opaque as above and unsigned with its range asserted, so that
// divisions and remainders by powers of two in the index arithmetic are shifts and masks.
template <int NT>
__device__ __forceinline__ unsigned opaque_tid(int tid) {
  const unsigned u = static_cast<unsigned>(opaque(tid));
  __builtin_assume(u < static_cast<unsigned>(NT));
  return u;
}

// pad() of an unsigned index.
__device__ __forceinline__ unsigned padu(unsigned e) { return e + (e >> 5); }

// f(e) for e = ut, ut + NT, ut + 2 NT, ... below N (ut < NT the thread index): unrolled,
// with a bound test only where N is not a multiple of NT.
template <int N, int NT, typename F>
__device__ __forceinline__ void for_strided(unsigned ut, F&& f) {
  constexpr int IT = (N + NT - 1) / NT;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    if (N % NT == 0 || e < static_cast<unsigned>(N)) f(e);
  }
}

// exp(DIR * 2 pi i j / R) for the twiddles inside the radix-8 and radix-16 butterflies.
template <int R, int DIR>
__device__ __forceinline__ float2 unit_root(int j) {
  // cos/sin of multiples of pi/8, exact to float rounding
  constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
  constexpr float C16[16] = {1.0f, c1, h, s1, 0.0f, -s1, -h, -c1, -1.0f, -c1, -h, -s1, 0.0f, s1, h, c1};
  constexpr float S16[16] = {0.0f, s1, h, c1, 1.0f, c1, h, s1, 0.0f, -s1, -h, -c1, -1.0f, -c1, -h, -s1};
  const int m = (j * (16 / R)) & 15;
  return make_float2(C16[m], DIR < 0 ? -S16[m] : S16[m]);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// 3-point DFT: y0 = a + b + c, y1,2 = a - (b + c)/2 -+ DIR-signed i (sqrt(3)/2)(b - c)
template <int DIR>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
  constexpr float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 t1 = cadd(b, c);
  const float2 t2 = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
  const float2 d = csub(b, c);
  // forward: y1 = t2 - i h d, y2 = t2 + i h d; inverse: the conjugate rotation
  const float2 r = DIR < 0 ? make_float2(h * d.y, -h * d.x) : make_float2(-h * d.y, h * d.x);
  a = cadd(a, t1);
  b = cadd(t2, r);
  c = csub(t2, r);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  const float2 a = cadd(x0, x2), b = csub(x0, x2);
  const float2 c = cadd(x1, x3), d = csub(x1, x3);
  // forward: y1 = b - i d, y3 = b + i d; inverse: the conjugate rotation
  const float2 jd = DIR < 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, jd);
  x3 = csub(b, jd);
}

// R-point DFT of v[0..R-1] in registers, in place.  R = 4 B: DFT_4 over the stride-B
// elements, twiddles w_R^(nB kA), then DFT_B over each group of B.  Output k = kA + 4 kB
// is left in v[out_slot<R>(k)] = v[kA B + kB] (no register shuffling; callers index the
// outputs through out_slot).
template <int R>
constexpr int out_slot(int k) {
  return R <= 4 ? k : (k % 4) * (R / 4) + k / 4;
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3<DIR>(v[0], v[1], v[2]);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else {
    constexpr int A = 4, B = R / 4;
#pragma unroll
    for (int nb = 0; nb < B; ++nb) dft4<DIR>(v[nb], v[nb + B], v[nb + 2 * B], v[nb + 3 * B]);
    // v[kA * B + nB] now holds DFT_A output kA of column nB
#pragma unroll
    for (int nb = 1; nb < B; ++nb)
#pragma unroll
      for (int ka = 1; ka < A; ++ka) v[ka * B + nb] = cmul(v[ka * B + nb], unit_root<R, DIR>(nb * ka));
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      if constexpr (B == 2) {
        dft2<DIR>(v[ka * B], v[ka * B + 1]);
      } else {
        dft4<DIR>(v[ka * B], v[ka * B + 1], v[ka * B + 2], v[ka * B + 3]);
      }
    }
  }
}

// Twiddles w^r (r = 1..R-1) from the table in global memory: only the bases w, w^2, w^4,
// w^8 are read (exact up to their FP32 rounding); applying them to v[r] forms the other
// powers as products of at most four of them.
template <int R>
__device__ __forceinline__ void read_twiddle_bases(float2* p, const float2* __restrict__ tw, int stride) {
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if ((1 << b) < R) p[b] = tw[(1 << b) * stride];
}

template <int R, int DIR>
__device__ __forceinline__ void apply_twiddle_bases(float2* v, const float2* p) {
#pragma unroll
  for (int r = 1; r < R; ++r) {
    float2 w = make_float2(1.0f, 0.0f);
    bool first = true;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (r & (1 << b)) {
        w = first ? p[b] : cmul(w, p[b]);
        first = false;
      }
    v[r] = DIR < 0 ? cmul(v[r], w) : cmulc(v[r], w);
  }
}


// Per-pass twiddle tables in LDS (TWL): the pass with span P and radix R reads
// T_P[(r - 1) P + k] = exp(-2 pi i r k / (P R)) for butterfly k = i mod P, so the lanes of
// a wave (consecutive k) read consecutive entries and every power is a single LDS read (no
// vector-memory issue, no products).  The tables of all passes of a length-N transform
// hold fewer than N entries in total.  stockham_pass reads them together with the data
// (before its barrier); this applies them from registers (w[r - 1] = T_P[(r - 1) P + k]).
template <int R, int DIR>
__device__ __forceinline__ void apply_twiddle_regs(float2* v, const float2* w) {
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = DIR < 0 ? cmul(v[r], w[r - 1]) : cmulc(v[r], w[r - 1]);
}

// One Stockham pass of radix R over NB transforms of length N, span P (product of the
// radices of the passes before it), executed by NTH threads.  The twiddles (read-only:
// the LDS tables, or the bases w, w^2, w^4, w^8 from the global table) are read before
// the pass's barrier together with the data, so that their latency is not added after it.
//
// Offsets.  With the base index B = off + t st + (i or j0) SI a multiple-of-32 apart from
// a value below the butterfly's span, pad(B + o_r) = pad(B) + pad(o_r) for the load
// offsets o_r = r (N/R) SI and the store offsets o_r = r P SI (N, R, P, SI powers of two),
// so pad(o_r) is a compile-time constant.
template <int N, int R, int P, int DIR, int NTH, int NB, bool TFAST, int SI, bool ALIGNED, bool TWL>
__device__ __forceinline__ void stockham_pass(float2* __restrict__ lds, int off, int st,
                                              const float2* __restrict__ tw, int tid) {
  constexpr int NBF = N / R;               // butterflies per transform
  constexpr int TOT = NBF * NB;            // butterflies per pass
  constexpr int BPT = (TOT + NTH - 1) / NTH;
  constexpr bool EXACT = (TOT % NTH) == 0;
  constexpr bool TWR = TWL && P > 1;  // twiddles read with the data
  constexpr bool TWG = !TWL && P > 1;  // global-table twiddle bases read with the data
  float2 v[BPT][R];
  float2 w[BPT][TWR ? R - 1 : 1];
  float2 wg[BPT][TWG ? 4 : 1];
  unsigned base[BPT], idx[BPT];
  const unsigned ut = opaque_tid<NTH>(tid);
  const unsigned uoff = static_cast<unsigned>(off), ust = static_cast<unsigned>(st);
#pragma unroll
  for (int s = 0; s < BPT; ++s) {
    const unsigned b = ut + s * NTH;
    unsigned t, i;
    if constexpr (TFAST) {
      t = b % NB;
      i = b / NB;
    } else {
      t = b / NBF;
      i = b % NBF;
    }
    base[s] = uoff + t * ust;
    idx[s] = i;
    if (EXACT || b < TOT) {
      if constexpr (ALIGNED) {
        const float2* src = lds + padu(base[s] + i * SI);
#pragma unroll
        for (int r = 0; r < R; ++r) v[s][r] = src[pad(r * NBF * SI)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[s][r] = lds[padu(base[s] + (i + r * NBF) * SI)];
      }
      if constexpr (TWR) {
        const float2* tp = tw + i % P;
#pragma unroll
        for (int r = 1; r < R; ++r) w[s][r - 1] = tp[(r - 1) * P];
      }
      if constexpr (TWG) read_twiddle_bases<R>(wg[s], tw, (i % P) * (N / (P * R)));
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < BPT; ++s) {
    const unsigned b = ut + s * NTH;
    if (EXACT || b < TOT) {
      const unsigned i = idx[s];
      const unsigned k = i % P;  // P is a compile-time constant (a shift and mask when a power of two)
      if constexpr (TWR)
        apply_twiddle_regs<R, DIR>(v[s], w[s]);
      else if constexpr (TWG)
        apply_twiddle_bases<R, DIR>(v[s], wg[s]);
      dft<R, DIR>(v[s]);
      const unsigned j0 = (i - k) * R + k;
      if constexpr (ALIGNED) {
        float2* dst = lds + padu(base[s] + j0 * SI);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[pad(r * P * SI)] = v[s][out_slot<R>(r)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) lds[padu(base[s] + (j0 + r * P) * SI)] = v[s][out_slot<R>(r)];
      }
    }
  }
  __syncthreads();
}

// Radix of the pass with span P.  Order 0: for N = 3 * 2^p a radix-3 pass first; then
// the remainder pass of the power-of-two part, then radix MAXR (8 or 16).  Order 1 (powers
// of two): radix MAXR first and the remainder pass last.
template <int N, int P, int MAXR, int ORD = 0>
constexpr int pass_radix() {
  if constexpr (ORD == 1) {
    constexpr int l = ilog2(N), m = ilog2(MAXR);
    return ((l % m) != 0 && P == (N >> (l % m))) ? (1 << (l % m)) : MAXR;
  } else {
    constexpr bool three = !is_pow2(N);
    if (three && P == 1) return 3;
    constexpr int l = ilog2(three ? N / 3 : N), m = ilog2(MAXR);
    if (P == (three ? 3 : 1) && (l % m) != 0) return 1 << (l % m);
    return MAXR;
  }
}

// Offset of the table of the pass with span PT in the per-pass tables of pass order ORD
// (and, for PT = N, their total size, always below N).
template <int N, int MAXR, int PT, int ORD = 0, int P = 1>
constexpr int tw_offset() {
  if constexpr (P >= PT || P >= N) {
    return 0;
  } else {
    constexpr int R = pass_radix<N, P, MAXR, ORD>();
    return (P > 1 ? (R - 1) * P : 0) + tw_offset<N, MAXR, PT, ORD, P * R>();
  }
}

// Build the per-pass tables of pass order ORD of a length-N transform in LDS from the full
// table tw[j] = exp(-2 pi i j / N) in global memory (callers have a barrier before use).
template <int N, int MAXR, int ORD = 0, int P = 1>
__device__ __forceinline__ void build_twiddles(float2* dst, const float2* __restrict__ tw, int tid, int nth) {
  if constexpr (P < N) {
    constexpr int R = pass_radix<N, P, MAXR, ORD>();
    if constexpr (P > 1) {
      constexpr int off = tw_offset<N, MAXR, P, ORD>();
      for (int j = tid; j < (R - 1) * P; j += nth) {
        const int r = j / P + 1, k = j % P;
        dst[off + j] = tw[r * k * (N / (P * R))];
      }
    }
    build_twiddles<N, MAXR, ORD, P * R>(dst, tw, tid, nth);
  }
}

// The passes with spans P .. STOP (exclusive) of pass order ORD.
template <int N, int P, int STOP, int ORD, int DIR, int NTH, int NB, bool TFAST, int SI, bool ALIGNED, int MAXR,
          bool TWL>
__device__ __forceinline__ void fft_passes(float2* lds, int off, int st, const float2* __restrict__ tw, int tid) {
  if constexpr (P < STOP) {
    constexpr int R = pass_radix<N, P, MAXR, ORD>();
    stockham_pass<N, R, P, DIR, NTH, NB, TFAST, SI, ALIGNED, TWL>(
        lds, off, st, TWL ? tw + tw_offset<N, MAXR, P, ORD>() : tw, tid);
    fft_passes<N, P * R, STOP, ORD, DIR, NTH, NB, TFAST, SI, ALIGNED, MAXR, TWL>(lds, off, st, tw, tid);
  }
}

// Full length-N transform of NB sequences in LDS; element i of transform t is at
// lds[pad(off + t * st + i * SI)].  ALIGNED asserts that off + t * st is always a multiple
// of 32 (see stockham_pass).  Callers must have a barrier between their last write of the
// data and this call; the call ends with a barrier.
template <int N, int DIR, int NTH, int NB, bool TFAST, int SI, bool ALIGNED, int MAXR = 16, bool TWL = true>
__device__ __forceinline__ void fft_lds(float2* lds, int off, int st, const float2* __restrict__ tw, int tid) {
  static_assert(fft_length_ok(N), "length 2^p or 3 * 2^p");
  static_assert(MAXR == 8 || MAXR == 16, "radix");
  // the compile-time offsets need power-of-two spans (see stockham_pass)
  static_assert(!ALIGNED || is_pow2(N), "aligned offsets need a power-of-two length");
  fft_passes<N, 1, N, 0, DIR, NTH, NB, TFAST, SI, ALIGNED, MAXR, TWL>(lds, off, st, tw, tid);
}

// Part of a transform: the passes of order ORD with spans P0 .. STOP (exclusive), for
// callers that fuse the first or the last pass into their own load or store.
template <int N, int P0, int STOP, int ORD, int DIR, int NTH, int NB, bool TFAST, int SI, bool ALIGNED, int MAXR,
          bool TWL>
__device__ __forceinline__ void fft_lds_part(float2* lds, int off, int st, const float2* __restrict__ tw, int tid) {
  static_assert(is_pow2(N) && (MAXR == 8 || MAXR == 16), "powers of two");
  static_assert(!ALIGNED || is_pow2(N), "aligned offsets need a power-of-two length");
  fft_passes<N, P0, STOP, ORD, DIR, NTH, NB, TFAST, SI, ALIGNED, MAXR, TWL>(lds, off, st, tw, tid);
}

}  // namespace fftlb
