// HIP kernels of one FFT-LB time step (gfx950).
//
// Spectral data layout ("row spectra").  A real plane g[ny][nx] is stored after its
// row transform as nx/2 complex columns per row: column 0 holds (Re G(0), Re G(nx/2))
// (the DC and Nyquist terms of a real row are real), columns 1..nx/2-1 hold G(kx).
// Columns are grouped in tiles of TW consecutive kx; a tile is stored as [y][TW], so a
// row kernel reads or writes TW * 8 bytes contiguous per tile and a column kernel
// reads a contiguous [ny][TW] block.  Element (y, kx) of a plane is at
//     (kx / TW) * ny * TW + y * TW + (kx % TW).
//
// Per time step (all derivatives by windowed FFT, Sec. 3.6):
//   k_col_conv_multi  one launch of two independent column passes: the y-parts v_y D_y f of
//                   the convection terms of some of the 24 populations with v_y != 0, formed
//                   from f (column FFT, i v_y k_m(ky) / ny, inverse column FFT) and left in
//                   real space;
//                   and a derivative pass of the macroscopic fields: 4 moment spectra -> 6
//                   y-derivative spectra (stage 1; launched with 16 of the populations),
//                   5 -> 3 divergence spectra (stage 2; with the other 8);
//   k_col_multi     the derivative passes by themselves (diagnostics);
//   k_rows_stage2   inverse row FFTs of the 11 derivatives, the pointwise closure of
//                   Eqs. (18)-(23), forward row FFTs of the 5 fields whose divergences the
//                   force needs, FP64 partial sums for the global diagnostics;
//   k_rows_collide  inverse row FFTs of the force divergences; the x-parts v_x D_x f of
//                   the 24 populations with v_x != 0 formed from f^n (forward row FFT, i k_x,
//                   inverse); the y-parts read in real space; equilibrium, force, explicit
//                   update, moments of f^{n+1} and their forward row FFTs (inputs of the next
//                   step).  With the finite-difference schemes the collide instead takes every
//                   convection spectrum from a column pass and writes the row spectra of f^{n+1}.
// Two real rows are transformed as one complex row (z = a + i b) and separated by
// Hermitian symmetry.
#pragma once
#include "fft_lds.hpp"
#include "model.hpp"

namespace fftlb {

// LDS allocation (in float2) of n padded elements (see fft_lds.hpp).
constexpr int lds_alloc(int n) { return padded_size(n); }

// Row-kernel geometry.  Each thread owns J sites of its row (J = 2, or 4 for 2048-point
// rows), a block holds RB rows (at least 64 threads), and row transforms are done four
// plane pairs at a time: a batch is 4 RB complex transforms of length NX, i.e. 4 J values
// per thread, so each pass is one butterfly of radix RADIX = 4 J per thread.  Radix 8
// (rather than 16) keeps the transform's registers small enough for two blocks per CU.
template <int NX>
struct RowGeom {
  static constexpr int J = NX >= 2048 ? 4 : 2;
  static constexpr int TPR = NX / J;
  static constexpr int RB = (TPR >= 64) ? 1 : 64 / TPR;
  static constexpr int NT = RB * TPR;
  static constexpr int NPB = 4;
  static constexpr int RADIX = 4 * J;
  static constexpr int LDS = lds_alloc(NPB * RB * NX);  // float2 elements of the data
  // Lengths whose pass sequence has a radix-2 remainder pass: the forward transforms run
  // it last and fuse it into the Hermitian store (saves one LDS round trip; fusing the
  // inverse's first pass into the load the same way was measured slower: its stride-2 LDS
  // writes conflict 4 ways).
  static constexpr bool FUSE_STORE = is_pow2(NX) && NX >= 16 && pass_radix<NX, 1, RADIX>() == 2;
  // after the data: per-pass twiddle tables of pass order 0, and of order 1 when fused
  static constexpr int LDS_TOTAL = LDS + (FUSE_STORE ? 2 : 1) * NX;
};

// Batch slot p of the row kernels starts at LDS element p * slot_stride (padded); RB NX is
// a multiple of 32, so pad(p RB NX + e) = p slot_stride + pad(e).
template <int NX>
constexpr int slot_stride() {
  static_assert((RowGeom<NX>::RB * NX) % 32 == 0, "batch slots start at multiples of 32");
  return pad(RowGeom<NX>::RB * NX);
}

// Per-pass twiddle tables of the row transforms in LDS after the data (callers have a
// barrier between this and the first transform).
template <int NX>
__device__ __forceinline__ const float2* row_twiddles(float2* lds, const float2* __restrict__ twx, int tid) {
  float2* dst = lds + RowGeom<NX>::LDS;
  build_twiddles<NX, RowGeom<NX>::RADIX, 0>(dst, twx, tid, RowGeom<NX>::NT);
  if constexpr (RowGeom<NX>::FUSE_STORE) build_twiddles<NX, RowGeom<NX>::RADIX, 1>(dst + NX, twx, tid, RowGeom<NX>::NT);
  return dst;
}

// The same for column transforms of length NY with largest radix R.
template <int NY, int R>
__device__ __forceinline__ const float2* col_twiddles(float2* dst, const float2* __restrict__ twy, int tid, int nth) {
  build_twiddles<NY, R>(dst, twy, tid, nth);
  return dst;
}

struct SpecGeom {
  int ny;       // column length
  int tw;       // tile width (power of two)
  int log2tw;
  __device__ __forceinline__ unsigned idx(unsigned y, unsigned k) const {
    return ((k >> log2tw) * ny + y) * tw + (k & (tw - 1));
  }
};

// Element i of an array at a wave-uniform base, addressed by a 32-bit byte offset (every
// plane is far below 4 GB): the access takes the base in scalar registers and needs no
// 64-bit address arithmetic per lane.  The base MUST be the same in every lane of the
// wave (it is taken from the first active lane; every caller passes kernel arguments
// plus uniform offsets); it is then made opaque in scalar registers so that the compiler
// cannot fold the address arithmetic of different planes into 64-bit per-lane sums.
using gbyte = __attribute__((address_space(1))) char;  // global-memory byte

template <typename T>
__device__ __forceinline__ T& elem(T* base, unsigned i) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(base);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(a >> 32));
  gbyte* b = (gbyte*)((static_cast<unsigned long long>(hi) << 32) | lo);
  asm("" : "+s"(b));
  return *(T*)(b + i * static_cast<unsigned>(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T& elem(const T* base, unsigned i) {
  return elem(const_cast<T*>(base), i);
}

// The populations f^n and f^{n+1} (and the low parts of a compensated state) are read once
// and written once per step by the collide: non-temporal accesses keep them from displacing,
// in the caches, the spectra that the column passes read right after the collide (measured
// at 1024^2: 0.2460 -> 0.2357 ms per step; making the spectra stores non-temporal as well was
// slower, 0.2396).
__device__ __forceinline__ float ld_stream(const float* base, unsigned i) {
  return __builtin_nontemporal_load(&elem(base, i));
}
__device__ __forceinline__ void st_stream(float* base, unsigned i, float v) {
  __builtin_nontemporal_store(v, &elem(base, i));
}

// Pointers into the workspace (and the caller's buffers for the init/set modes).
struct Planes {
  float* f;          // [33][ny][nx]
  float* flo;        // [33][ny][nx] low parts of a compensated state f = f + flo (null: FP32 state)
  float2* sf;        // [32] row spectra of f_1..f_32 (in place: convection spectra after the column pass)
  float2* sm;        // [4]  row spectra of rho, ux, uy, T
  float2* s1;        // [6]  stage-1 y-derivative spectra
  float2* s2i;       // [5]  stage-2 input spectra
  float2* s2o;       // [3]  stage-2 output spectra: B^x, B^y, G
  float* macro;      // [4][ny][nx] rho, ux, uy, T (real)
  float* cpl;        // [ny][nx] coefficient C of Eq. (22)
  const float2* twx; // row twiddles, nx entries
  const float* kapx; // windowed k_x, nx/2 entries
  double* part_d;    // [blocks][6] stage-2 partials: mass, px, py, energy, max|u|, nonfinite
  float* part_f;     // [blocks][2] residual-pass partials: max |D.(rho u)|, nonfinite
  int nx, ny;
  long plane;        // nx * ny
  SpecGeom sg;
};

// The workspace pointers of an instance are never null (the host fills every one):
// asserting it lets the compiler drop the null tests of the batch helpers, whose
// branches would otherwise split the address arithmetic of the spectral accesses.
__device__ __forceinline__ void assume_planes(const Planes& P) {
  __builtin_assume(P.f != nullptr);
  __builtin_assume(P.sf != nullptr);
  __builtin_assume(P.sm != nullptr);
  __builtin_assume(P.s1 != nullptr);
  __builtin_assume(P.s2i != nullptr);
  __builtin_assume(P.s2o != nullptr);
  __builtin_assume(P.macro != nullptr);
  __builtin_assume(P.cpl != nullptr);
}

// Multiplier kinds of the multi-output column pass.
enum : int {
  MK_NONE = 0,
  MK_IKX = 1,   // i k_x
  MK_IKY = 2,   // i k_y
  MK_KXX = 3,   // -k_x^2
  MK_KYY = 4,   // -k_y^2
  MK_KXY = 5,   // -k_x k_y
  MK_LAP = 6,   // -(k_x^2 + k_y^2)
};

// One derivative group of a column pass: nin input planes, nout output planes, each output
// the sum over inputs p of kind[o][p] applied to input p.  Planes are indices into an
// instance's spectral block (the moment, stage-1 and stage-2 spectra, contiguous).
struct ColGroup {
  int in[3];
  int out[6];
  int nin, nout;
  int kind[6][3];
};

struct ColLaunch {
  ColGroup g[4];
};

// Kernel arguments are passed by value: pointers inside kernel arguments are known to
// address global memory, so they compile to global loads and stores (pointers read from a
// descriptor in device memory would be flat accesses, which also hold up the LDS waits).
// A launch covers up to kRowSlots (row kernels) or kColSlots (column kernels) instances of
// one grid size; blockIdx.y (row and convection kernels) or blockIdx.z (derivative column
// passes) selects the slot.  A single solver is a launch of one slot.
constexpr int kRowSlots = 8;
constexpr int kColSlots = 32;

struct RowArgs {
  Planes P[kRowSlots];
  Model M[kRowSlots];
  int id[kRowSlots];   // instance ids, for the retirement flags
  const int* state;    // per-instance retired flags of a batch (null: none)
};

struct ColInst {
  float2* spec;        // convection: the 32 population spectra; derivatives: the spectral block
  const float2* twy;   // column twiddles, ny entries
  const float* kapx;   // windowed k_x, nx/2 entries
  const float* kapy;   // windowed k_y, ny entries
  int nx, tw, id;
  float scale;         // 1 / (nx ny)
  const float2* freal; // f_0..f_32 in real space, each plane read as [ny][nx/2] pairs of sites
  float yscale;        // 1 / ny
};

struct ColArgs {
  ColInst c[kColSlots];
  const int* state;
};

// Inputs of the init (rho0, ux0, uy0, T0) and set-state (f) modes of the collide kernel.
struct Inputs {
  const float* a[4];
};

// True when the instance of a slot has been retired by the batch poll.
__device__ __forceinline__ bool retired(const int* state, int id) { return state && state[id]; }

// ---------------------------------------------------------------------------
// Block helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool nonfinite(float x) { return !(fabsf(x) <= 3.402823466e38f); }

// x as a rounded FP32 value: keeps the compiler from fusing the multiply that produced x
// into a later add (the moments of f^eq must be those of the stored f, exactly as when
// the same f is loaded back by the set-state mode).
__device__ __forceinline__ float rounded(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Row groups: thread -> (row within block rl, lane within row lt).  Sites are addressed
// from the first site of the block's rows (a wave-uniform base): site(j) = rl NX + x(j).
template <int NX>
struct RowThread {
  static constexpr int TPR = RowGeom<NX>::TPR;
  unsigned rl, lt;
  __device__ __forceinline__ explicit RowThread(int tid) {
    const unsigned u = static_cast<unsigned>(tid);
    __builtin_assume(u < static_cast<unsigned>(RowGeom<NX>::NT));
    rl = u / TPR;
    lt = u % TPR;
  }
  __device__ __forceinline__ unsigned x(int j) const { return lt + j * TPR; }
  __device__ __forceinline__ unsigned site(int j) const { return rl * NX + x(j); }
  // LDS element of site x(j) in batch slot `slot` (slots start at multiples of 32)
  __device__ __forceinline__ unsigned at(int slot, int j) const {
    constexpr unsigned SL = slot_stride<NX>();
    if constexpr (TPR % 32 == 0)
      return slot * SL + padu(rl * NX + lt) + j * pad(TPR);
    else
      return slot * SL + padu(rl * NX + x(j));
  }
};

// A batch of up to four plane pairs: pair p transforms z = a + i b.  Each of a and b is a
// row-spectral linear combination of at most two stored spectra, term = c m(kx) S with
//   m = 1 (TERM_ONE), i k_x (TERM_IKX) or -k_x^2 (TERM_KXX),
// k_x the windowed wavenumber (zero at kx = 0 and at the Nyquist column packed with it).
// A derivative along x alone never needs a column transform: it is a row-spectral product.
enum : int { TERM_ONE = 0, TERM_IKX = 1, TERM_KXX = 2 };

// Which terms are present is kept in flags of their own (`on`), so that where a batch is
// built from set_term calls the presence is a compile-time fact and the loads need no
// runtime tests.
template <int NP>
struct PairBatch {
  const float2* s[NP][2][2];  // [pair][a, b][term]
  float c[NP][2][2];
  int kind[NP][2][2];
  bool on[NP][2][2];          // term present
};

// A batch with no terms (pairs left without terms load as zero).
template <int NP>
__device__ __forceinline__ PairBatch<NP> empty_batch() {
  PairBatch<NP> r;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        r.s[p][h][t] = nullptr;
        r.c[p][h][t] = 1.0f;
        r.kind[p][h][t] = TERM_ONE;
        r.on[p][h][t] = false;
      }
  return r;
}

// Term t of side h (0 = a, 1 = b) of pair p: c m(kx) s, s a valid spectrum (never null).
template <int NP>
__device__ __forceinline__ void set_term(PairBatch<NP>& b, int p, int h, int t, const float2* s, float c, int kind) {
  b.s[p][h][t] = s;
  b.c[p][h][t] = c;
  b.kind[p][h][t] = kind;
  b.on[p][h][t] = true;
}

// a[p] + i b[p] as they are; a null pointer is an absent side (tested at run time).
template <int NP>
__device__ __forceinline__ PairBatch<NP> plain_batch(const float2* const (&a)[NP], const float2* const (&b)[NP]) {
  PairBatch<NP> r = empty_batch<NP>();
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    r.s[p][0][0] = a[p];
    r.s[p][1][0] = b[p];
    r.on[p][0][0] = a[p] != nullptr;
    r.on[p][1][0] = b[p] != nullptr;
  }
  return r;
}

template <int NP>
struct PairBatchOut {
  float2* a[NP];
  float2* b[NP];
  bool hb[NP];           // b[p] present
};

// Loading a batch is split in two so that callers can issue the global loads early:
// rows_fetch_batch reads the raw spectral values of every present term (and k_x) into
// registers, rows_put_batch combines them and writes the LDS slots.
template <int NX, int NP>
struct BatchFetch {
  static constexpr int IT = (RowGeom<NX>::RB * (NX / 2) + RowGeom<NX>::NT - 1) / RowGeom<NX>::NT;
  float2 v[IT][NP][2][2];
  float kx[IT];
};

template <int NX, int NP>
__device__ __forceinline__ BatchFetch<NX, NP> rows_fetch_batch(const PairBatch<NP>& in, const SpecGeom& sg,
                                                               const float* __restrict__ kapx, int row0, int tid) {
  constexpr unsigned H = NX / 2;
  constexpr int RB = RowGeom<NX>::RB;
  constexpr int NT = RowGeom<NX>::NT;
  using F = BatchFetch<NX, NP>;
  F r;
  const unsigned ut = opaque_tid<NT>(tid);
#pragma unroll
  for (int it = 0; it < F::IT; ++it) {
    const unsigned e = ut + it * NT;
    if (RB * H % NT == 0 || e < RB * H) {
      const unsigned rl = e / H, k = e % H;
      const unsigned gi = sg.idx(row0 + rl, k);
      r.kx[it] = elem(kapx, k);
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (in.on[p][h][t]) r.v[it][p][h][t] = elem(in.s[p][h][t], gi);
    }
  }
  return r;
}

// Value of one side of a pair from its fetched terms.  The k_x table is zero at column 0
// (both of its packed entries, DC and Nyquist, have k_x = 0), so the packed column needs
// no case of its own.
template <int NX, int NP>
__device__ __forceinline__ float2 combo_value(const PairBatch<NP>& in, const BatchFetch<NX, NP>& F, int it, int p,
                                              int h) {
  float2 acc = make_float2(0.0f, 0.0f);
  const float kx = F.kx[it];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (!in.on[p][h][t]) continue;
    const float2 v = F.v[it][p][h][t];
    const float c = in.c[p][h][t];
    const int kd = in.kind[p][h][t];
    if (kd == TERM_ONE) {
      acc.x += c * v.x;
      acc.y += c * v.y;
    } else if (kd == TERM_IKX) {
      acc.x -= c * kx * v.y;
      acc.y += c * kx * v.x;
    } else {
      const float m = -c * kx * kx;
      acc.x += m * v.x;
      acc.y += m * v.y;
    }
  }
  return acc;
}

// LDS slot p <- Z(k) = A(k) + i B(k), k = 0..NX-1, for every row of the block, from the
// fetched packed half spectra; Hermitian completion of the upper half.  The packed column
// k = 0 (A = (A(0), A(H)), B likewise, all real) is handled by masks and selects rather
// than a branch, so that all accesses of the batch stay in one basic block.
template <int NX, int NP>
__device__ __forceinline__ void rows_put_batch(float2* lds, const PairBatch<NP>& in, const BatchFetch<NX, NP>& F,
                                               int tid) {
  constexpr unsigned H = NX / 2;
  constexpr int RB = RowGeom<NX>::RB;
  constexpr int NT = RowGeom<NX>::NT;
  constexpr int SL = slot_stride<NX>();
  const unsigned ut = opaque_tid<NT>(tid);
#pragma unroll
  for (int it = 0; it < BatchFetch<NX, NP>::IT; ++it) {
    const unsigned e = ut + it * NT;
    if (RB * H % NT == 0 || e < RB * H) {
      const unsigned rl = e / H, k = e % H;
      const bool k0 = k == 0;
      const float m = k0 ? 0.0f : 1.0f;
      const unsigned z = rl * NX;
      const unsigned l0 = padu(z + k), l1 = padu(z + (k0 ? H : NX - k));
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const float2 a = combo_value(in, F, it, p, 0);
        const float2 b = combo_value(in, F, it, p, 1);
        float2* L = lds + p * SL;
        // k > 0: Z(k) = a + i b, Z(N - k) = conj(a) + i conj(b);
        // k = 0: Z(0) = A(0) + i B(0) = (a.x, b.x), Z(H) = (a.y, b.y)
        L[l0] = make_float2(fmaf(-m, b.y, a.x), fmaf(m, a.y, b.x));
        L[l1] = make_float2(k0 ? a.y : a.x + b.y, k0 ? b.y : b.x - a.y);
      }
    }
  }
}

// Both steps at once.  kapx (nx/2 windowed k_x values, zero at column 0) must always be a
// valid table.
template <int NX, int NP>
__device__ __forceinline__ void rows_load_batch(float2* lds, const PairBatch<NP>& in, const SpecGeom& sg,
                                                const float* __restrict__ kapx, int row0, int tid) {
  rows_put_batch<NX, NP>(lds, in, rows_fetch_batch<NX, NP>(in, sg, kapx, row0, tid), tid);
}

// Packed half spectra of A = Re z and B = Im z from the forward transforms Z in LDS slots.
template <int NX, int NP>
__device__ __forceinline__ void rows_store_batch(const float2* lds, const PairBatchOut<NP>& out,
                                                 const SpecGeom& sg, int row0, int tid) {
  constexpr unsigned H = NX / 2;
  constexpr int RB = RowGeom<NX>::RB;
  constexpr int NT = RowGeom<NX>::NT;
  constexpr int SL = slot_stride<NX>();
  const unsigned ut = opaque_tid<NT>(tid);
  for_strided<RB * H, NT>(ut, [&](unsigned e) {
    const unsigned rl = e / H, k = e % H;
    const bool k0 = k == 0;
    const unsigned z = rl * NX;
    const unsigned l0 = padu(z + k), l1 = padu(z + (k0 ? H : NX - k));
    const unsigned gi = sg.idx(row0 + rl, k);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const float2 Z = lds[p * SL + l0], W = lds[p * SL + l1];
      // k > 0: A = (Z + conj W) / 2, B = (Z - conj W) / (2i) with W = Z(N - k);
      // k = 0 (W = Z(H)): A = (Z.x, W.x), B = (Z.y, W.y)
      const float2 A = make_float2(k0 ? Z.x : 0.5f * (Z.x + W.x), k0 ? W.x : 0.5f * (Z.y - W.y));
      const float2 B = make_float2(k0 ? Z.y : 0.5f * (Z.y + W.y), k0 ? W.y : 0.5f * (W.x - Z.x));
      elem(out.a[p], gi) = A;
      if (out.hb[p]) elem(out.b[p], gi) = B;
    }
  });
}

// Store of the packed half spectra with the last (radix-2, span H) forward pass fused in:
// the thread for spectral column k (0 <= k <= Q = H/2) computes the butterflies i = k and
// i = H - k (inputs i, i + H, twiddle w_i = tw_last[i]; outputs X(i) = y(i) + w y(i + H)
// and X(i + H) = y(i) - w y(i + H)), which yield X at k, N - k, H - k and H + k, and
// separates columns k and H - k.  k = Q is its own partner (both stores agree).  The
// thread of the packed column k = 0 takes butterfly Q as its partner (in range, unused),
// and its partner store goes to column 0 first and is overwritten by the right value.
// No branches: all stores of the batch stay in one basic block.
template <int NX, int NP>
__device__ __forceinline__ void rows_store_batch_r2(const float2* lds, const PairBatchOut<NP>& out, const SpecGeom& sg,
                                                    const float2* tw_last, int row0, int tid) {
  constexpr unsigned H = NX / 2, Q = H / 2, W = Q + 1;
  constexpr int RB = RowGeom<NX>::RB;
  constexpr int NT = RowGeom<NX>::NT;
  constexpr int SL = slot_stride<NX>();
  const unsigned ut = opaque_tid<NT>(tid);
  for_strided<RB * W, NT>(ut, [&](unsigned e) {
    const unsigned rl = e / W, k = e % W;
    const bool k0 = k == 0;
    const unsigned k2 = k0 ? Q : H - k;
    const unsigned z = rl * NX;
    const unsigned lk = padu(z + k), lkh = padu(z + k + H);
    const unsigned lk2 = padu(z + k2), lk2h = padu(z + k2 + H);
    const float2 w1 = tw_last[k], w2 = tw_last[k2];
    const unsigned gi = sg.idx(row0 + rl, k);
    const unsigned gi2 = k0 ? gi : sg.idx(row0 + rl, k2);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const float2* L = lds + p * SL;
      const float2 t = cmul(L[lkh], w1), u = L[lk];
      const float2 Xk = cadd(u, t), Xkh = csub(u, t);     // X(k), X(k + H)
      const float2 t2 = cmul(L[lk2h], w2), u2 = L[lk2];
      const float2 Xk2 = cadd(u2, t2);                    // X(H - k)
      const float2 Xn = k0 ? Xk : csub(u2, t2);           // X(N - k) (k = 0: X(0))
      // column H - k from X(H - k) and X(N - (H - k)) = X(H + k)
      const float2 A2 = make_float2(0.5f * (Xk2.x + Xkh.x), 0.5f * (Xk2.y - Xkh.y));
      const float2 B2 = make_float2(0.5f * (Xk2.y + Xkh.y), 0.5f * (Xkh.x - Xk2.x));
      // column k; for k = 0 the packed (X(0), X(H)): A = (X(0).x, X(H).x), B = (X(0).y, X(H).y)
      const float2 A = make_float2(0.5f * (Xk.x + Xn.x), k0 ? Xkh.x : 0.5f * (Xk.y - Xn.y));
      const float2 B = make_float2(0.5f * (Xk.y + Xn.y), k0 ? Xkh.y : 0.5f * (Xn.x - Xk.x));
      elem(out.a[p], gi2) = A2;
      if (out.hb[p]) elem(out.b[p], gi2) = B2;
      elem(out.a[p], gi) = A;
      if (out.hb[p]) elem(out.b[p], gi) = B;
    }
  });
}

// Inverse row transforms of the NP slots in LDS (after a barrier); afterwards slot p holds
// a_p(x) + i b_p(x).  twx: the per-pass LDS tables (TWL) or the global table.
template <int NX, int NP, bool TWL = true>
__device__ __forceinline__ void rows_inverse_fft(float2* lds, const float2* twx, int tid) {
  using G = RowGeom<NX>;
  constexpr bool AL = is_pow2(NX) && (NX % 32 == 0);
  fft_lds<NX, +1, G::NT, NP * G::RB, false, 1, AL, G::RADIX, TWL>(lds, 0, NX, twx, tid);
}

// Load and inverse row transforms of a batch.
template <int NX, int NP, bool TWL = true>
__device__ __forceinline__ void rows_inverse_batch(float2* lds, const PairBatch<NP>& in, const SpecGeom& sg,
                                                   const float2* twx, const float* kapx, int row0, int tid) {
  rows_load_batch<NX, NP>(lds, in, sg, kapx, row0, tid);
  __syncthreads();
  rows_inverse_fft<NX, NP, TWL>(lds, twx, tid);
}

// Forward row transforms of slots already written (unsynchronised) and store of the packed
// half spectra.  Ends with a barrier so the LDS can be reused.
template <int NX, int NP, bool TWL = true>
__device__ __forceinline__ void rows_forward_batch(float2* lds, const PairBatchOut<NP>& out, const SpecGeom& sg,
                                                   const float2* twx, int row0, int tid) {
  using G = RowGeom<NX>;
  constexpr bool AL = is_pow2(NX) && (NX % 32 == 0);
  __syncthreads();
  if constexpr (G::FUSE_STORE) {
    // pass order 1 (radix-2 remainder last), its tables after those of order 0
    const float2* tw1 = TWL ? twx + NX : twx;
    fft_lds_part<NX, 1, NX / 2, 1, -1, G::NT, NP * G::RB, false, 1, AL, G::RADIX, TWL>(lds, 0, NX, tw1, tid);
    // twiddles of the last pass: T[k] = exp(-2 pi i k / N), or the global table itself
    const float2* tw_last = TWL ? tw1 + tw_offset<NX, G::RADIX, NX / 2, 1>() : twx;
    rows_store_batch_r2<NX, NP>(lds, out, sg, tw_last, row0, tid);
  } else {
    fft_lds<NX, -1, G::NT, NP * G::RB, false, 1, AL, G::RADIX, TWL>(lds, 0, NX, twx, tid);
    rows_store_batch<NX, NP>(lds, out, sg, row0, tid);
  }
  __syncthreads();
}

// Windowed k_x of signed FFT bin m of a length-NX row (odd in m, zero at the Nyquist bin),
// from kapx[0 .. NX/2 - 1].
template <int NX>
__device__ __forceinline__ float kx_of_bin(const float* __restrict__ kapx, unsigned m) {
  constexpr unsigned H = NX / 2;
  return m < H ? elem(kapx, m) : m == H ? 0.0f : -elem(kapx, NX - m);
}

// Slot `slot` of the row batch holds the forward transforms Z of complex rows z = a + i b
// (a, b real): multiply bin m by i k_x(m) / NX, so that the inverse transform gives
// D_x a + i D_x b (the multiplier is odd in m and zero at the Nyquist bin, so the two real
// rows stay apart).  Each thread reads and writes its own elements (no barrier inside).
template <int NX>
__device__ __forceinline__ void rows_dx_multiply(float2* lds, int slot, const float* __restrict__ kapx, int tid) {
  constexpr int RB = RowGeom<NX>::RB, NT = RowGeom<NX>::NT;
  constexpr float s = 1.0f / NX;
  float2* L = lds + slot * slot_stride<NX>();
  const unsigned ut = opaque_tid<NT>(tid);
  for_strided<RB * NX, NT>(ut, [&](unsigned e) {
    const float k = kx_of_bin<NX>(kapx, e % NX) * s;
    const float2 v = L[padu(e)];
    L[padu(e)] = make_float2(-k * v.y, k * v.x);
  });
}

// The same after all passes but the last (radix-2, span H) of pass order 1: the thread of
// butterfly k (0 <= k < H) forms X(k) = u + w_k t and X(k + H) = u - w_k t from u = Z(k),
// t = Z(k + H) and multiplies both.
template <int NX>
__device__ __forceinline__ void rows_dx_multiply_r2(float2* lds, int slot, const float2* tw_last,
                                                    const float* __restrict__ kapx, int tid) {
  constexpr unsigned H = NX / 2;
  constexpr int RB = RowGeom<NX>::RB, NT = RowGeom<NX>::NT;
  constexpr float s = 1.0f / NX;
  float2* L = lds + slot * slot_stride<NX>();
  const unsigned ut = opaque_tid<NT>(tid);
  for_strided<RB * H, NT>(ut, [&](unsigned e) {
    const unsigned rl = e / H, k = e % H;
    const unsigned z = rl * NX;
    const float2 u = L[padu(z + k)], t = cmul(L[padu(z + k + H)], tw_last[k]);
    const float2 x0 = cadd(u, t), x1 = csub(u, t);
    const float k0 = elem(kapx, k) * s;                          // bin k
    const float k1 = k == 0 ? 0.0f : -elem(kapx, H - k) * s;      // bin k + H (Nyquist for k = 0)
    L[padu(z + k)] = make_float2(-k0 * x0.y, k0 * x0.x);
    L[padu(z + k + H)] = make_float2(-k1 * x1.y, k1 * x1.x);
  });
}

// Forward row transforms of slots 0 .. NS - 1 written (unsynchronised), each multiplied by
// i k_x / NX in place (rows_dx_multiply): after an inverse transform they hold D_x of their
// two real rows.  No barrier at the end (callers have one before the next transform).
template <int NX, int NS>
__device__ __forceinline__ void rows_dx_forward(float2* lds, const float2* twx, const float* __restrict__ kapx,
                                                int tid) {
  using G = RowGeom<NX>;
  constexpr bool AL = is_pow2(NX) && (NX % 32 == 0);
  __syncthreads();
  if constexpr (G::FUSE_STORE) {
    const float2* tw1 = twx + NX;
    fft_lds_part<NX, 1, NX / 2, 1, -1, G::NT, NS * G::RB, false, 1, AL, G::RADIX, true>(lds, 0, NX, tw1, tid);
    const float2* tw_last = tw1 + tw_offset<NX, G::RADIX, NX / 2, 1>();
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) rows_dx_multiply_r2<NX>(lds, sl, tw_last, kapx, tid);
  } else {
    fft_lds<NX, -1, G::NT, NS * G::RB, false, 1, AL, G::RADIX, true>(lds, 0, NX, twx, tid);
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) rows_dx_multiply<NX>(lds, sl, kapx, tid);
  }
}

// ---------------------------------------------------------------------------
// Column kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  // Consecutive logical blocks land on the same XCD (blocks are dealt round-robin to 8 XCDs),
  // so column tiles that share cache lines share an L2.
  if (nblocks % 8) return b;
  return (b % 8) * (nblocks / 8) + b / 8;
}

// Convection with the spectral derivative: the term v.grad f = v_x D_x f + v_y D_y f of a
// population splits by axis (the 2D multiplier i (v_x k_m(kx) + v_y k_m(ky)) is a sum of
// one-axis multipliers).  The column pass forms the y-part v_y D_y f of each of the 24
// moving populations with v_y != 0 (directions i != 1, 5) from f itself, two real columns
// at a time as one complex column (the multiplier is odd in k_y and zero at the Nyquist row,
// so the two stay apart), and leaves it in real space, row-major, in the population's
// spectral plane; the collide forms the x-parts from f^n along its rows.  No population is
// row-transformed between the kernels.
__device__ __forceinline__ int conv_column_plane(int j) {
  // j = 0..23 -> population q - 1 = 8 k + i - 1 with i - 1 in {1, 2, 3, 5, 6, 7}
  const int k = j / 6, r = j % 6;
  return 8 * k + (r < 3 ? r + 1 : r + 2);
}

// Pairs of the collide's row transforms.  Finite-difference schemes (every convection
// spectrum from a column pass): direction offsets (i - 1) (0,1) (2,3) (4,5) (6,7) of a speed
// group, spectra stored and read.  Spectral derivative: the x-derivative pairs (0,4) (1,3)
// (5,7) of the six directions with v_x != 0, formed from f^n in the collide.
constexpr int pair_dir(bool direct, int p, int h) { return direct ? (p == 0 ? 4 * h : 4 * p - 3 + 2 * h) : 2 * p + h; }

// Tile b of nblocks (planes pfirst.. of the 24, (nx/2)/CW column tiles each) of one
// instance: v_y D_y f of population p + 1 (f plane p + 1 read as [ny][nx/2] pairs of sites)
// into spectral plane p, both row-major.
template <int NY, int CW, int NT, int R>
__device__ __forceinline__ void col_conv_body(const ColInst& In, float2* lds, int b, int nblocks, int pfirst) {
  const float2* twy = In.twy;
  const float* __restrict__ kapy = In.kapy;
  const int nx = In.nx;
  const int tid = threadIdx.x;
  const unsigned ut = static_cast<unsigned>(tid);
  __builtin_assume(ut < static_cast<unsigned>(NT));
  twy = col_twiddles<NY, R>(lds + lds_alloc(NY * CW), twy, tid, NT);
  const int nsub = (nx / 2) / CW;
  b = xcd_remap(b, nblocks);
  const int p = conv_column_plane(pfirst + b / nsub), sub = b % nsub;
  const unsigned c0 = sub * CW;
  const unsigned stride = static_cast<unsigned>(nx / 2);
  float2* g = In.spec + (long)p * (nx / 2) * NY + c0;
  const float2* src = In.freal + (long)(p + 1) * (nx / 2) * NY + c0;
  // element e of the block is (y, c) = (e / CW, e % CW).  The k_y of the thread's elements
  // are read with the data, so that their latency is not added after the forward transform.
  constexpr int IT = (NY * CW + NT - 1) / NT;
  constexpr bool FULL = (NY * CW) % NT == 0;
  float kyv[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    kyv[i] = (FULL || e < static_cast<unsigned>(NY * CW)) ? elem(kapy, e / CW) : 0.0f;
  }
  const float vys = c_vel.vy[p + 1] * In.yscale;
  for_strided<NY * CW, NT>(ut, [&](unsigned e) {
    const unsigned y = e / CW, c = e % CW;
    lds[padu(e)] = elem(src, y * stride + c);
  });
  __syncthreads();
  fft_lds<NY, -1, NT, CW, true, CW, is_pow2(NY) && (NY * CW % 32 == 0), R>(lds, 0, 1, twy, tid);
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    if (FULL || e < static_cast<unsigned>(NY * CW)) {
      const float m = vys * kyv[i];
      const float2 v = lds[padu(e)];
      lds[padu(e)] = make_float2(-m * v.y, m * v.x);
    }
  }
  __syncthreads();
  fft_lds<NY, +1, NT, CW, true, CW, is_pow2(NY) && (NY * CW % 32 == 0), R>(lds, 0, 1, twy, tid);
  for_strided<NY * CW, NT>(ut, [&](unsigned e) {
    const unsigned y = e / CW, c = e % CW;
    elem(g, y * stride + c) = lds[padu(e)];
  });
}


// Convection by one of the finite-difference schemes of Sec. 3.1 (Lax-Wendroff, Eq. (ML-);
// MLW1 = LW + R3, MLW2 = LW + R3 + R4, Eqs. (R3), (R4=)), applied per axis and summed.  On
// the periodic grid each stencil is a multiplication of the spectrum, so the scheme's
// update of f is applied exactly (up to rounding) in the same column passes: with
// c = v dt / d (the CFL number of the axis), s = sin(theta), e = cos(theta) - 1 and
// theta = k d, the stencils of one axis add to f^n the multiple
//   -i c s [1 - r3 (1 - c^2) e / 3] + c^2 e [1 + r4 (1 - c^2) e / 2]
// of each mode (the CD term -i c s, the LW term c^2 e, R3 = i c (1 - c^2) s e / 3 and
// R4 = c^2 (1 - c^2) e^2 / 2), i.e. the convection term D = -(that) / dt, which the collide
// multiplies by -dt as for the spectral derivative.  The nine-point stencils of the NPS scheme
// (Sec. 3.1, A = 1/3, B = 1/12) have the cross-axis symbols
//   D_x = i s_x (2 + cos theta_y) / (3 dx),  D_y = i s_y (2 + cos theta_x) / (3 dy),
// so their convection term times dt is i [c_x s_x (3 + e_y) + c_y s_y (3 + e_x)] / 3.
struct SchemeInst {
  float2* spec;            // the 32 population spectra (in place)
  const float2* twy;       // column twiddles, ny entries
  const float2* scx;       // (sin theta, cos theta - 1) of k_x = 0..nx/2-1, theta = 2 pi k_x / nx
  const float2* scy;       // the same of k_y = 0..ny-1
  int nx, tw, id;
  float cfx, cfy;          // dt / dx, dt / dy
  float r3, r4;            // 1 where the R3 / R4 terms are on, else 0
  float sdt;               // 1 / (nx ny dt)
  int nps;                 // 1: the NPS stencils instead of the LW family
};

constexpr int kSchemeSlots = 8;
struct SchemeArgs {
  SchemeInst c[kSchemeSlots];
  const int* state;
};

// D of one axis times dt for CFL number c at (s, e): (real, imaginary).
__device__ __forceinline__ float2 scheme_axis(float c, float2 se, float r3, float r4) {
  const float w = 1.0f - c * c;
  const float im = c * se.x * (1.0f - r3 * w * se.y * (1.0f / 3.0f));
  const float re = -c * c * se.y * (1.0f + r4 * w * se.y * 0.5f);
  return make_float2(re, im);
}

// dt D at (s, e) of k_x and of k_y: (real, imaginary).
__device__ __forceinline__ float2 scheme_symbol(const SchemeInst& In, float cx, float cy, float2 sx, float2 sy) {
  if (In.nps) return make_float2(0.0f, (cx * sx.x * (3.0f + sy.y) + cy * sy.x * (3.0f + sx.y)) * (1.0f / 3.0f));
  const float2 a = scheme_axis(cx, sx, In.r3, In.r4), b = scheme_axis(cy, sy, In.r3, In.r4);
  return make_float2(a.x + b.x, a.y + b.y);
}

// (s, e) of the x Nyquist wavenumber, theta = pi
__device__ __forceinline__ float2 nyquist_se() { return make_float2(0.0f, -2.0f); }

// Product of a packed column's spectrum with two multipliers.  Column 0 of the row spectra
// holds Z = A + i B with A, B the (real) DC and Nyquist columns of the x transform; their y
// spectra are A^ = (Z^(ky) + conj Z^(-ky)) / 2 and i B^ = (Z^(ky) - conj Z^(-ky)) / 2, and the
// result is m_a A^ + i m_b B^ (m_a at k_x = 0, m_b at the x Nyquist wavenumber).  z = Z^(ky),
// w = Z^(-ky).
__device__ __forceinline__ float2 packed_product(float2 ma, float2 mb, float2 z, float2 w) {
  const float2 wc = make_float2(w.x, -w.y);
  const float2 a = cmul(ma, cadd(z, wc)), b = cmul(mb, csub(z, wc));
  return make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
}

// Tile b of nblocks (all 32 moving populations, (nx/2)/CW column tiles each): forward
// column FFT, multiplication by D(kx, ky) (scaled by 1/(nx ny)), inverse column FFT.  The
// packed column 0 takes packed_product (the scheme's multipliers differ between its DC and
// Nyquist halves), which reads the mirror element -ky: every product is formed in
// registers before any is written back.
template <int NY, int CW, int NT, int R>
__device__ __forceinline__ void col_scheme_body(const SchemeInst& In, float2* lds, int b, int nblocks) {
  const float2* twy = In.twy;
  const int nx = In.nx;
  const unsigned tw = In.tw;
  const int tid = threadIdx.x;
  const unsigned ut = static_cast<unsigned>(tid);
  __builtin_assume(ut < static_cast<unsigned>(NT));
  twy = col_twiddles<NY, R>(lds + lds_alloc(NY * CW), twy, tid, NT);
  const int nsub = (nx / 2) / CW;
  b = xcd_remap(b, nblocks);
  const int p = b / nsub, sub = b % nsub;
  const unsigned c0 = sub * CW;
  float2* g = In.spec + (long)p * (nx / 2) * NY + (long)(c0 / tw) * NY * tw + (c0 % tw);
  const float vx = c_vel.vx[p + 1], vy = c_vel.vy[p + 1];
  const float cx = vx * In.cfx, cy = vy * In.cfy;
  static_assert(NT % CW == 0, "a thread keeps one column");
  const unsigned col = c0 + ut % CW;
  const float2 sx = elem(In.scx, col);
  const bool packed = col == 0;
  for_strided<NY * CW, NT>(ut, [&](unsigned e) {
    const unsigned y = e / CW, c = e % CW;
    lds[padu(e)] = elem(g, y * tw + c);
  });
  __syncthreads();
  fft_lds<NY, -1, NT, CW, true, CW, is_pow2(NY) && (NY * CW % 32 == 0), R>(lds, 0, 1, twy, tid);
  const float sdt = In.sdt;
  constexpr int IT = (NY * CW + NT - 1) / NT;
  constexpr bool FULL = (NY * CW) % NT == 0;
  float2 res[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    if (!(FULL || e < static_cast<unsigned>(NY * CW))) continue;
    const unsigned y = e / CW, c = e % CW;
    const float2 sy = elem(In.scy, y);
    const float2 m = scheme_symbol(In, cx, cy, sx, sy);
    const float2 z = lds[padu(e)];
    float2 r = cmul(m, z);
    if (packed) {
      const float2 w = lds[padu(((NY - y) % NY) * CW + c)];
      r = packed_product(m, scheme_symbol(In, cx, cy, nyquist_se(), sy), z, w);
    }
    res[i] = make_float2(r.x * sdt, r.y * sdt);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    if (FULL || e < static_cast<unsigned>(NY * CW)) lds[padu(e)] = res[i];
  }
  __syncthreads();
  fft_lds<NY, +1, NT, CW, true, CW, is_pow2(NY) && (NY * CW % 32 == 0), R>(lds, 0, 1, twy, tid);
  for_strided<NY * CW, NT>(ut, [&](unsigned e) {
    const unsigned y = e / CW, c = e % CW;
    elem(g, y * tw + c) = lds[padu(e)];
  });
}

template <int NY, int CW, int NT, int R>
__global__ __launch_bounds__(NT) void k_col_conv_scheme(SchemeArgs A) {
  const SchemeInst& In = A.c[blockIdx.y];
  if (retired(A.state, In.id)) return;
  extern __shared__ float2 lds[];
  col_scheme_body<NY, CW, NT, R>(In, lds, blockIdx.x, gridDim.x);
}

// Column pass of derivative groups: forward column FFTs of the nin input spectra, then
// each output the linear combination sum_p m_op(kx, ky) X_p, inverse column FFTs, store.
//
// LDS layout: transform-contiguous (as in the row kernels): column c of plane slot p is
// transform t = p CW + c, its element y at lds[pad(t NY + y)], so that the transforms of
// all nin inputs (and later of all nout outputs) are one batched call whose passes walk
// consecutive butterflies of one transform.  The combination is done in place by the
// thread that owns (y, c) of every slot.  Group shapes (nin, nout) are compile-time in the
// body; the kernel dispatches on them.
constexpr int kMultiSlots = 3;

__device__ __forceinline__ float2 mk_apply(int kd, float kx, float ky, float2 v) {
  // m v for the multiplier kinds: i k_x, i k_y (imaginary), -k_x^2, -k_y^2, -k_x k_y,
  // -(k_x^2 + k_y^2) (real)
  const float ai = kd == MK_IKX ? kx : kd == MK_IKY ? ky : 0.0f;
  const float ar = kd == MK_KXX   ? -kx * kx
                 : kd == MK_KYY   ? -ky * ky
                 : kd == MK_KXY   ? -kx * ky
                 : kd == MK_LAP   ? -(kx * kx + ky * ky)
                                  : 0.0f;
  return make_float2(ar * v.x - ai * v.y, ar * v.y + ai * v.x);
}

template <int NY, int CW, int NT, int R, int NIN, int NOUT>
__device__ __forceinline__ void col_multi_body(const ColInst& In, const ColGroup& G, float2* lds, const float2* twy,
                                               unsigned ut, int tid, unsigned c0, long off) {
  static_assert(NIN <= kMultiSlots && NOUT <= kMultiSlots, "group shape");
  constexpr int BLK = NY * CW;  // elements (y, c) of one plane
  // transforms start at multiples of 32 (NY a power of two >= 32): compile-time offsets
  constexpr bool AL = is_pow2(NY) && NY % 32 == 0;
  const unsigned tw = In.tw;
  const long hp = (long)(In.nx / 2) * NY;  // complex values per spectral plane
  const float scale = In.scale;
  // the wavenumbers of the thread's elements in the combination (e = c NY + y), read with
  // the data so that their latency is not added after the forward transforms
  constexpr int IT = (BLK + NT - 1) / NT;
  constexpr bool FULL = BLK % NT == 0;
  float kxv[IT], kyv[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    const bool in = FULL || e < static_cast<unsigned>(BLK);
    kxv[i] = in ? elem(In.kapx, c0 + e / NY) : 0.0f;
    kyv[i] = in ? elem(In.kapy, e % NY) : 0.0f;
  }
  // global side: consecutive lanes take consecutive columns of a row (e = y CW + c)
#pragma unroll
  for (int p = 0; p < NIN; ++p) {
    const float2* g = In.spec + G.in[p] * hp + off;
    for_strided<BLK, NT>(ut, [&](unsigned e) {
      const unsigned y = e / CW, c = e % CW;
      lds[padu((p * CW + c) * NY + y)] = elem(g, y * tw + c);
    });
  }
  __syncthreads();
  fft_lds<NY, -1, NT, NIN * CW, false, 1, AL, R>(lds, 0, NY, twy, tid);
  int kd[NOUT][NIN];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int p = 0; p < NIN; ++p) kd[o][p] = G.kind[o][p];
  // combination: consecutive lanes take consecutive rows of a column (e = c NY + y)
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned e = ut + i * NT;
    if (!(FULL || e < static_cast<unsigned>(BLK))) continue;
    const unsigned c = e / NY, y = e % NY;
    const float kx = kxv[i], ky = kyv[i];
    float2 x[NIN];
#pragma unroll
    for (int p = 0; p < NIN; ++p) x[p] = lds[padu((p * CW + c) * NY + y)];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int p = 0; p < NIN; ++p) acc = cadd(acc, mk_apply(kd[o][p], kx, ky, x[p]));
      lds[padu((o * CW + c) * NY + y)] = make_float2(acc.x * scale, acc.y * scale);
    }
  }
  __syncthreads();
  fft_lds<NY, +1, NT, NOUT * CW, false, 1, AL, R>(lds, 0, NY, twy, tid);
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float2* g = In.spec + G.out[o] * hp + off;
    for_strided<BLK, NT>(ut, [&](unsigned e) {
      const unsigned y = e / CW, c = e % CW;
      elem(g, y * tw + c) = lds[padu((o * CW + c) * NY + y)];
    });
  }
}

// Group shapes with a compiled body (every group the solver builds has one of them).
__host__ __device__ constexpr bool multi_shape_ok(int nin, int nout) {
  return (nin == 1 && (nout == 1 || nout == 2)) || (nin == 2 && (nout == 1 || nout == 3)) || (nin == 3 && nout == 2);
}

// Column tile b of ntiles ((nx/2)/CW) of group G of one instance.
template <int NY, int CW, int NT, int R>
__device__ __forceinline__ void col_multi_tile(const ColInst& In, const ColGroup& G, float2* lds, int b, int ntiles) {
  const int tid = threadIdx.x;
  const unsigned ut = static_cast<unsigned>(tid);
  __builtin_assume(ut < static_cast<unsigned>(NT));
  const float2* twy = col_twiddles<NY, R>(lds + lds_alloc(kMultiSlots * NY * CW), In.twy, tid, NT);
  const unsigned tw = In.tw;
  const unsigned c0 = xcd_remap(b, ntiles) * CW;
  const long off = (long)(c0 / tw) * NY * tw + (c0 % tw);
  switch (G.nin * 4 + G.nout) {
    case 1 * 4 + 1: col_multi_body<NY, CW, NT, R, 1, 1>(In, G, lds, twy, ut, tid, c0, off); break;
    case 1 * 4 + 2: col_multi_body<NY, CW, NT, R, 1, 2>(In, G, lds, twy, ut, tid, c0, off); break;
    case 2 * 4 + 1: col_multi_body<NY, CW, NT, R, 2, 1>(In, G, lds, twy, ut, tid, c0, off); break;
    case 2 * 4 + 3: col_multi_body<NY, CW, NT, R, 2, 3>(In, G, lds, twy, ut, tid, c0, off); break;
    case 3 * 4 + 2: col_multi_body<NY, CW, NT, R, 3, 2>(In, G, lds, twy, ut, tid, c0, off); break;
    default: break;  // not built by the host (multi_shape_ok)
  }
}

template <int NY, int CW, int NT, int R>
__global__ __launch_bounds__(NT, 4) void k_col_multi(ColArgs A, ColLaunch L) {
  const ColInst& In = A.c[blockIdx.z];
  if (retired(A.state, In.id)) return;
  extern __shared__ float2 lds[];
  col_multi_tile<NY, CW, NT, R>(In, L.g[blockIdx.y], lds, blockIdx.x, gridDim.x);
}

// Convection by the flux-limiter scheme of Sec. 3.1: each population is convected along its
// own lattice direction e (the characteristic line; A = 1 along an axis, sqrt(2) along a
// diagonal) with CFL number c = v_k dt / (A dr):
//   C = v_k / (A dr) [F_{J+1/2} - F_{J-1/2}],  F_{J+1/2} = f_J + (1 - c)/2 psi(theta_J) (f_{J+1} - f_J),
// theta_J = (f_J - f_{J-1}) / (f_{J+1} - f_J), J +- 1 the nodes at J +- e.  The MCD limiter
// (0 for theta <= 0, 2 theta up to 1/3, (1 + theta)/2 up to 3, 2 beyond) times the difference
// it multiplies is, with a = f_J - f_{J-1}, b = f_{J+1} - f_J: 0 when a b <= 0, otherwise
// sign(b) min(2|a|, |a + b|/2, 2|b|) (the same values without the division; zero when b = 0).
// The limiter makes the scheme nonlinear, so it runs in real space (k_conv_fl, stencil.hpp):
// one thread per site and population, writing the real convection planes that row transforms
// then take to spectra.
struct FlArgs {
  const float* f;          // [33][ny][nx] f^n (the high part of a compensated state)
  float* out;              // [32][ny][nx] convection terms of the moving populations, times 1/nx
                           // (the unnormalised forward and inverse row transforms they pass
                           // through on the way to the collide multiply by nx)
  int nx, ny, id;
  float cf;                // dt / dr
  float rdr;               // 1 / dr
};

struct FlBatch {
  FlArgs c[kSchemeSlots];
  const int* state;
};

__device__ __forceinline__ float mcd_limited(float a, float b) {
  if (!(a * b > 0.0f)) return 0.0f;
  const float m = fminf(fminf(2.0f * fabsf(a), 0.5f * fabsf(a + b)), 2.0f * fabsf(b));
  return copysignf(m, b);
}


// Derivative groups with the nine-point stencils of the NPS scheme (Sec. 3.1): A = 1/3,
// B = 1/12 for the first derivative, E = 2/3, F = 1/6 for the Laplacian.  On the periodic grid
// each stencil is a multiplication of the spectrum; with s = sin(theta), e = cos(theta) - 1 of
// each axis (theta = k d, dx = dy = d):
//   D_x = i s_x (3 + e_y) / (3 dx),   D_y = i s_y (3 + e_x) / (3 dy),
//   Lap = [2 (e_x + e_y) + (2/3) e_x e_y] / d^2,
// and the group kinds map onto them: i k_x -> D_x, i k_y -> D_y, -k_x^2 -> D_x D_x,
// -k_y^2 -> D_y D_y, -k_x k_y -> D_x D_y, -(k_x^2 + k_y^2) -> Lap.  One column per block:
// these groups run by themselves (not inside the convection launches).
struct NpsInst {
  float2* spec;            // the spectral block
  const float2* twy;       // column twiddles, ny entries
  const float2* scx;       // (sin theta, cos theta - 1) of k_x = 0..nx/2-1
  const float2* scy;       // the same of k_y = 0..ny-1
  int nx, tw, id;
  float rdx, rdy;          // 1 / dx, 1 / dy
  float scale;             // 1 / (nx ny)
};

struct NpsArgs {
  NpsInst c[kSchemeSlots];
  const int* state;
};

__device__ __forceinline__ float2 nps_multiplier(int kd, float2 sx, float2 sy, float rdx, float rdy) {
  const float dx = sx.x * (3.0f + sy.y) * (1.0f / 3.0f) * rdx;  // D_x = i dx
  const float dy = sy.x * (3.0f + sx.y) * (1.0f / 3.0f) * rdy;  // D_y = i dy
  const float lap = (2.0f * (sx.y + sy.y) + (2.0f / 3.0f) * sx.y * sy.y) * (rdx * rdy);
  const float ai = kd == MK_IKX ? dx : kd == MK_IKY ? dy : 0.0f;
  const float ar = kd == MK_KXX   ? -dx * dx
                 : kd == MK_KYY   ? -dy * dy
                 : kd == MK_KXY   ? -dx * dy
                 : kd == MK_LAP   ? lap
                                  : 0.0f;
  return make_float2(ar, ai);
}

template <int NY, int NT, int R, int NIN, int NOUT>
__device__ __forceinline__ void col_nps_body(const NpsInst& In, const ColGroup& G, float2* lds, const float2* twy,
                                             unsigned ut, int tid, unsigned col) {
  static_assert(NIN <= kMultiSlots && NOUT <= kMultiSlots, "group shape");
  constexpr bool AL = is_pow2(NY) && NY % 32 == 0;
  const unsigned tw = In.tw;
  const long hp = (long)(In.nx / 2) * NY;
  const long off = (long)(col / tw) * NY * tw + (col % tw);
#pragma unroll
  for (int p = 0; p < NIN; ++p) {
    const float2* g = In.spec + G.in[p] * hp + off;
    for_strided<NY, NT>(ut, [&](unsigned y) { lds[padu(p * NY + y)] = elem(g, y * tw); });
  }
  __syncthreads();
  fft_lds<NY, -1, NT, NIN, false, 1, AL, R>(lds, 0, NY, twy, tid);
  int kd[NOUT][NIN];
#pragma unroll
  for (int o = 0; o < NOUT; ++o)
#pragma unroll
    for (int p = 0; p < NIN; ++p) kd[o][p] = G.kind[o][p];
  const float2 sx = elem(In.scx, col);
  const bool packed = col == 0;  // the block's column: (DC, Nyquist) of the x transform
  constexpr int IT = (NY + NT - 1) / NT;
  constexpr bool FULL = NY % NT == 0;
  // products into registers first: the packed column reads the mirror element -ky
  float2 res[IT][NOUT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned y = ut + i * NT;
    if (!(FULL || y < static_cast<unsigned>(NY))) continue;
    const float2 sy = elem(In.scy, y);
    float2 x[NIN], w[NIN];
#pragma unroll
    for (int p = 0; p < NIN; ++p) {
      x[p] = lds[padu(p * NY + y)];
      w[p] = packed ? lds[padu(p * NY + (NY - y) % NY)] : x[p];
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int p = 0; p < NIN; ++p) {
        const float2 m = nps_multiplier(kd[o][p], sx, sy, In.rdx, In.rdy);
        acc = cadd(acc, packed ? packed_product(m, nps_multiplier(kd[o][p], nyquist_se(), sy, In.rdx, In.rdy), x[p],
                                                w[p])
                               : cmul(m, x[p]));
      }
      res[i][o] = make_float2(acc.x * In.scale, acc.y * In.scale);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const unsigned y = ut + i * NT;
    if (!(FULL || y < static_cast<unsigned>(NY))) continue;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) lds[padu(o * NY + y)] = res[i][o];
  }
  __syncthreads();
  fft_lds<NY, +1, NT, NOUT, false, 1, AL, R>(lds, 0, NY, twy, tid);
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    float2* g = In.spec + G.out[o] * hp + off;
    for_strided<NY, NT>(ut, [&](unsigned y) { elem(g, y * tw) = lds[padu(o * NY + y)]; });
  }
}

// Group shapes of the NPS groups: those of the windowed groups and (1, 3).
__host__ __device__ constexpr bool nps_shape_ok(int nin, int nout) {
  return multi_shape_ok(nin, nout) || (nin == 1 && nout == 3);
}

template <int NY, int NT, int R>
__global__ __launch_bounds__(NT) void k_col_nps(NpsArgs A, ColLaunch L) {
  const NpsInst& In = A.c[blockIdx.z];
  if (retired(A.state, In.id)) return;
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const unsigned ut = static_cast<unsigned>(tid);
  __builtin_assume(ut < static_cast<unsigned>(NT));
  const float2* twy = col_twiddles<NY, R>(lds + lds_alloc(kMultiSlots * NY), In.twy, tid, NT);
  const unsigned col = xcd_remap(blockIdx.x, In.nx / 2);
  const ColGroup& G = L.g[blockIdx.y];
  switch (G.nin * 4 + G.nout) {
    case 1 * 4 + 1: col_nps_body<NY, NT, R, 1, 1>(In, G, lds, twy, ut, tid, col); break;
    case 1 * 4 + 2: col_nps_body<NY, NT, R, 1, 2>(In, G, lds, twy, ut, tid, col); break;
    case 1 * 4 + 3: col_nps_body<NY, NT, R, 1, 3>(In, G, lds, twy, ut, tid, col); break;
    case 2 * 4 + 1: col_nps_body<NY, NT, R, 2, 1>(In, G, lds, twy, ut, tid, col); break;
    case 2 * 4 + 3: col_nps_body<NY, NT, R, 2, 3>(In, G, lds, twy, ut, tid, col); break;
    case 3 * 4 + 2: col_nps_body<NY, NT, R, 3, 2>(In, G, lds, twy, ut, tid, col); break;
    default: break;  // not built by the host (nps_shape_ok)
  }
}

// Convection tiles of planes pfirst.. and a derivative pass (of ngroups groups) in one
// launch: the first nc blocks of a slot run the convection tiles, the ngroups nt blocks
// after them the derivative tiles (CWM columns each, nt = (nx/2)/CWM tiles per group) with the
// convection pass's block size and radix.  The two passes are independent: the
// latency-bound derivative tiles, dispatched last, run in the slots that the convection
// tiles free as that pass drains (measured faster than dispatching them first).
struct ConvMultiArgs {
  ColArgs a;                 // the convection pass's instances (population spectra)
  float2* mspec[kColSlots];  // the spectral block of each instance
};

template <int NY, int CW, int NT, int R, int CWM>
__global__ __launch_bounds__(NT, 4) void k_col_conv_multi(ConvMultiArgs A, ColLaunch L, int ngroups, int pfirst) {
  const ColInst& In = A.a.c[blockIdx.y];
  if (retired(A.a.state, In.id)) return;
  extern __shared__ float2 lds[];
  const int nt = (In.nx / 2) / CWM;
  const int nm = ngroups * nt, nc = gridDim.x - nm;
  const int b = blockIdx.x;
  if (b >= nc) {
    ColInst Im = In;
    Im.spec = A.mspec[blockIdx.y];
    col_multi_tile<NY, CWM, NT, R>(Im, L.g[(b - nc) / nt], lds, (b - nc) % nt, nt);
  } else {
    col_conv_body<NY, CW, NT, R>(In, lds, b, nc, pfirst);
  }
}

// ---------------------------------------------------------------------------
// Row kernels
// ---------------------------------------------------------------------------

// Stage 2: derivatives at the sites, closure of Eqs. (18)-(23), forward row transforms of
// P1 = S + Lxx, P2 = Lxy, P3 = S + Lyy, gx, gy; C to its plane; diagnostics partials.
// NPS: all 11 derivatives come from the column pass (the nine-point stencils couple the
// axes), s1 = [rx, ry, lap, dxux, dyux, dxuy] and the five planes after the spectral block's
// 18, [dyuy, thx, thy, Tx, Ty].
template <int NX, bool NPS = false>
__device__ __forceinline__ void rows_stage2(const Planes& P, const Model& M, int blk) {
  extern __shared__ float2 lds[];
  using G = RowGeom<NX>;
  constexpr int J = G::J;
  const int tid = threadIdx.x;
  // twiddles from the global table here: an LDS copy would cost this kernel one of its
  // four blocks per CU
  const float2* twx = P.twx;
  const RowThread<NX> rt(tid);
  const int row0 = blk * G::RB;
  const long rb = (long)row0 * NX;  // first site of the block's rows
  const float* mac = P.macro + rb;
  const long hp = P.plane / 2;

  float rho[J], ux[J], uy[J], T[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const unsigned s = rt.site(j);
    rho[j] = elem(mac, s);
    ux[j] = elem(mac + P.plane, s);
    uy[j] = elem(mac + 2 * P.plane, s);
    T[j] = elem(mac + 3 * P.plane, s);
  }
  // The 11 stage-1 derivatives d = rx, ry, lap, dxux, dyux, dxuy, dyuy, thx, thy, Tx, Ty.
  // x-derivatives are row-spectral products of the moment spectra R, Ux, Uy, Th (scaled by
  // 1/nx for the unnormalised inverse row transform); the column pass supplied
  // s1 = [D_y rho, D_yy rho, D_y ux, D_y uy, D_y theta, D_y T], already normalised.
  float d[11][J];
  {
    const float inx = 1.0f / P.nx;
    const float2 *R = P.sm, *Ux = P.sm + hp, *Uy = P.sm + 2 * hp, *Th = P.sm + 3 * hp;
    const float2* s1 = P.s1;
    PairBatch<4> b = empty_batch<4>();
    PairBatch<2> b2 = empty_batch<2>();
    if constexpr (NPS) {
      const float2* sn = s1 + 14 * hp;  // plane 18 of the spectral block
      set_term(b, 0, 0, 0, s1, 1.0f, TERM_ONE);               // rx
      set_term(b, 0, 1, 0, s1 + hp, 1.0f, TERM_ONE);          // ry
      set_term(b, 1, 0, 0, s1 + 2 * hp, 1.0f, TERM_ONE);      // lap
      set_term(b, 1, 1, 0, s1 + 3 * hp, 1.0f, TERM_ONE);      // dxux
      set_term(b, 2, 0, 0, s1 + 4 * hp, 1.0f, TERM_ONE);      // dyux
      set_term(b, 2, 1, 0, sn + hp, 1.0f, TERM_ONE);          // thx
      set_term(b, 3, 0, 0, s1 + 5 * hp, 1.0f, TERM_ONE);      // dxuy
      set_term(b, 3, 1, 0, sn, 1.0f, TERM_ONE);               // dyuy
      set_term(b2, 0, 0, 0, sn + 2 * hp, 1.0f, TERM_ONE);     // thy
      set_term(b2, 0, 1, 0, sn + 3 * hp, 1.0f, TERM_ONE);     // Tx
      set_term(b2, 1, 0, 0, sn + 4 * hp, 1.0f, TERM_ONE);     // Ty
    } else {
      set_term(b, 0, 0, 0, R, inx, TERM_IKX);                 // rx
      set_term(b, 0, 1, 0, s1, 1.0f, TERM_ONE);               // ry
      set_term(b, 1, 0, 0, R, inx, TERM_KXX);                 // lap = D_xx rho + D_yy rho
      set_term(b, 1, 0, 1, s1 + hp, 1.0f, TERM_ONE);
      set_term(b, 1, 1, 0, Ux, inx, TERM_IKX);                // dxux
      set_term(b, 2, 0, 0, s1 + 2 * hp, 1.0f, TERM_ONE);      // dyux
      set_term(b, 2, 1, 0, Ux, inx, TERM_KXX);                // thx = D_x(D_x ux + D_y uy)
      set_term(b, 2, 1, 1, s1 + 3 * hp, 1.0f, TERM_IKX);
      set_term(b, 3, 0, 0, Uy, inx, TERM_IKX);                // dxuy
      set_term(b, 3, 1, 0, s1 + 3 * hp, 1.0f, TERM_ONE);      // dyuy
      set_term(b2, 0, 0, 0, s1 + 4 * hp, 1.0f, TERM_ONE);     // thy
      set_term(b2, 0, 1, 0, Th, inx, TERM_IKX);               // Tx
      set_term(b2, 1, 0, 0, s1 + 5 * hp, 1.0f, TERM_ONE);     // Ty
    }
    // both batches are read at once; the second waits in registers during the first's
    // transforms
    const BatchFetch<NX, 4> f1 = rows_fetch_batch<NX, 4>(b, P.sg, P.kapx, row0, tid);
    const BatchFetch<NX, 2> f2 = rows_fetch_batch<NX, 2>(b2, P.sg, P.kapx, row0, tid);
    rows_put_batch<NX, 4>(lds, b, f1, tid);
    __syncthreads();
    rows_inverse_fft<NX, 4, false>(lds, twx, tid);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float2 v = lds[rt.at(0, j)];
      d[0][j] = v.x;
      d[1][j] = v.y;
      v = lds[rt.at(1, j)];
      d[2][j] = v.x;
      d[3][j] = v.y;
      v = lds[rt.at(2, j)];
      d[4][j] = v.x;
      d[7][j] = v.y;
      v = lds[rt.at(3, j)];
      d[5][j] = v.x;
      d[6][j] = v.y;
    }
    __syncthreads();
    rows_put_batch<NX, 2>(lds, b2, f2, tid);
    __syncthreads();
    rows_inverse_fft<NX, 2, false>(lds, twx, tid);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float2 v = lds[rt.at(0, j)];
      d[8][j] = v.x;
      d[9][j] = v.y;
      d[10][j] = lds[rt.at(1, j)].x;
    }
    __syncthreads();
  }

  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  float umax = 0.0f;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const float r = rho[j], t = T[j];
    const float rx = d[0][j], ry = d[1][j], lap = d[2][j];
    const float dxux = d[3][j], dyux = d[4][j], dxuy = d[5][j], dyuy = d[6][j];
    const float thx = d[7][j], thy = d[8][j], Tx = d[9][j], Ty = d[10][j];
    const float theta = dxux + dyuy;
    const float Mg = M.K + M.H * t;
    const float rT = r * t;
    const float Pw = rT / (1.0f - M.b * r) - M.a * r * r;
    const float S = Pw - rT - M.zeta * theta;
    const float grad2 = rx * rx + ry * ry;
    const float iso = r * M.K * (rx * Tx + ry * Ty) / t - Mg * (r * lap + 0.5f * grad2);
    const float Lxx = Mg * rx * rx + iso;
    const float Lyy = Mg * ry * ry + iso;
    const float Lxy = Mg * rx * ry;
    // slots: 0 = (S + Lxx, Lxy), 1 = (S + Lyy, gx), 2 = (gy, 0)
    lds[rt.at(0, j)] = make_float2(S + Lxx, Lxy);
    lds[rt.at(1, j)] = make_float2(S + Lyy, 2.0f * M.q * rT * Tx);
    lds[rt.at(2, j)] = make_float2(2.0f * M.q * rT * Ty, 0.0f);
    const float lam_du = Lxx * dxux + Lxy * dxuy + Lxy * dyux + Lyy * dyuy;
    const float cubic = rx * (dxux * rx + dxuy * ry) + ry * (dyux * rx + dyuy * ry);
    const float num = (Pw - rT) * theta + lam_du - M.zeta * theta * theta + M.a * r * r * theta +
                      M.K * (-0.5f * grad2 * theta - r * (rx * thx + ry * thy) - cubic);
    const float C = num / (2.0f * rT * t);
    elem(P.cpl + rb, rt.site(j)) = C;
    const float u2 = ux[j] * ux[j] + uy[j] * uy[j];
    const double e = (double)rT - (double)M.a * r * r + 0.5 * (double)M.K * grad2 + 0.5 * (double)r * u2;
    acc[0] += r;
    acc[1] += (double)r * ux[j];
    acc[2] += (double)r * uy[j];
    acc[3] += e;
    umax = fmaxf(umax, sqrtf(u2));
    bad |= nonfinite(r) | nonfinite(t) | nonfinite(u2) | nonfinite(C);
  }
  // forward row transforms of the five fields whose divergences the force needs
  PairBatchOut<3> o{{P.s2i, P.s2i + 2 * hp, P.s2i + 4 * hp}, {P.s2i + hp, P.s2i + 3 * hp, nullptr}, {true, true, false}};
  rows_forward_batch<NX, 3, false>(lds, o, P.sg, twx, row0, tid);

  // block reduction of the diagnostics (fixed order: deterministic)
  __shared__ double red_d[16][4];
  __shared__ float red_f[16][2];
  const int wave = tid / 64, lane = tid % 64;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = wave_sum(acc[i]);
  umax = wave_max(umax);
  const float badf = wave_max(bad ? 1.0f : 0.0f);
  if (lane == 0) {
    for (int i = 0; i < 4; ++i) red_d[wave][i] = acc[i];
    red_f[wave][0] = umax;
    red_f[wave][1] = badf;
  }
  __syncthreads();
  if (tid == 0) {
    constexpr int NW = (G::NT + 63) / 64;
    double sm[4] = {0, 0, 0, 0};
    float um = 0.0f, bd = 0.0f;
    for (int w = 0; w < NW; ++w) {
      for (int i = 0; i < 4; ++i) sm[i] += red_d[w][i];
      um = fmaxf(um, red_f[w][0]);
      bd = fmaxf(bd, red_f[w][1]);
    }
    double* out = P.part_d + 6 * (long)blk;
    for (int i = 0; i < 4; ++i) out[i] = sm[i];
    out[4] = um;
    out[5] = bd;
  }
}

template <int NX, bool NPS = false>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_stage2(RowArgs A) {
  const int s = blockIdx.y;
  if (retired(A.state, A.id[s])) return;
  assume_planes(A.P[s]);
  rows_stage2<NX, NPS>(A.P[s], A.M[s], blockIdx.x);
}

enum : int { MODE_STEP = 0, MODE_INIT = 1, MODE_SET = 2 };

// Collision, force and update (MODE_STEP), or f := f^eq(inputs) (MODE_INIT), or f := input
// (MODE_SET); then moments of the new f and forward row transforms of f_1..f_32 and of
// rho, ux, uy, T for the next step.  The 32 moving populations go in four rounds of one
// speed group (8 populations) each: 4 pair transforms per round (XCOL), or with the spectral
// derivative the 3 x-derivative pairs (see below).
//
// COMP: the state is compensated, f = hi + lo with the low parts in P.flo: the update adds
// every increment exactly (relax_update_comp), the moments add the sums of the low parts,
// and the row transforms (the next convection terms) take hi; INIT and SET zero lo.
//
// XCOL: the convection spectra of all 32 moving populations come from a column pass (the
// finite-difference schemes, k_col_conv_scheme); otherwise the x-parts of the convection
// terms are formed here from f^n and the y-parts are read in real space.
template <int NX, int MODE, bool COMP = false, bool XCOL = false>
__device__ __forceinline__ void rows_collide(const Planes& P, const Model& M, const Inputs& in, int blk) {
  extern __shared__ float2 lds[];
  using G = RowGeom<NX>;
  constexpr int J = G::J;
  constexpr int GPR = G::NPB / 4;   // speed groups per round
  const int tid = threadIdx.x;
  const float2* twx = row_twiddles<NX>(lds, P.twx, tid);
  const RowThread<NX> rt(tid);
  const int row0 = blk * G::RB;
  const long rb = (long)row0 * NX;  // first site of the block's rows
  float* mac = P.macro + rb;
  const long hp = P.plane / 2;

  // Moving populations: each round covers one speed group (q = 1 + 8k .. 8 + 8k for group
  // k, directions i = 1..8).  With XCOL, four pair transforms of the group (pair_dir): the
  // inverse transforms of their convection spectra (consecutive planes q0 - 1 .. q0 + 6) at
  // the start, the forward transforms of f^{n+1} (the next spectra) at the end.  With the
  // spectral derivative (DIRECT) no population spectra exist: the convection term is
  // v_x D_x f + v_y D_y f, the y-parts come in real space from the column pass, and the x-parts
  // of the six directions with v_x != 0 are formed here from f^n: three pairs z = f_a + i f_b
  // (pair_dir) transformed forward and multiplied by i k_x / nx at the end of the previous
  // round (the first group's after the force transforms) and inverse-transformed at the
  // start of the round.
  static_assert(GPR == 1, "one speed group per round");
  constexpr bool DIRECT = !XCOL;
  constexpr int NPR = G::NPB;  // pair transforms per round with XCOL
  constexpr int NX3 = 3;       // x-derivative pairs per round with DIRECT
  auto conv_batch = [&](int rd) {
    const int q0 = 1 + 8 * rd;
    const float2* S = P.sf + (long)(q0 - 1) * hp;
    PairBatch<NPR> in = empty_batch<NPR>();
#pragma unroll
    for (int p = 0; p < NPR; ++p)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int d = pair_dir(DIRECT, p, h);
        set_term(in, p, h, 0, S + d * hp, 1.0f, TERM_ONE);
      }
    return in;
  };
  // With J = 2 the loads of a round are issued ahead: the next round's convection spectra
  // during this round's forward transforms (the first round's during the force
  // transforms), f^n of the round's populations during its inverse transforms (16
  // registers each).
  constexpr bool PREF = MODE == MODE_STEP && J == 2;
  if constexpr (COMP) __builtin_assume(P.flo != nullptr);
  BatchFetch<NX, NPR> cf;
  Site st[J];
  if constexpr (MODE == MODE_STEP) {
    PairBatch<2> b2 = empty_batch<2>();
    set_term(b2, 0, 0, 0, P.s2o, 1.0f, TERM_ONE);           // B^x
    set_term(b2, 0, 1, 0, P.s2o + hp, 1.0f, TERM_ONE);      // B^y
    set_term(b2, 1, 0, 0, P.s2o + 2 * hp, 1.0f, TERM_ONE);  // G
    const BatchFetch<NX, 2> f2 = rows_fetch_batch<NX, 2>(b2, P.sg, P.kapx, row0, tid);
    // the site's moments and C, read while the force spectra are transformed
    float mr[J], mux[J], muy[J], mt[J], mc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const unsigned s = rt.site(j);
      mr[j] = elem(mac, s);
      mux[j] = elem(mac + P.plane, s);
      muy[j] = elem(mac + 2 * P.plane, s);
      mt[j] = elem(mac + 3 * P.plane, s);
      mc[j] = elem(P.cpl + rb, s);
    }
    if constexpr (PREF && !DIRECT) cf = rows_fetch_batch<NX, NPR>(conv_batch(0), P.sg, P.kapx, row0, tid);
    rows_put_batch<NX, 2>(lds, b2, f2, tid);
    __syncthreads();
    rows_inverse_fft<NX, 2>(lds, twx, tid);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float2 bxy = lds[rt.at(0, j)];
      const float gd = lds[rt.at(1, j)].x;
      const float r = mr[j], t = mt[j];
      site_init(st[j], r, mux[j], muy[j], t);
      const float irT = 1.0f / (r * t);
      const float cc = mc[j] + 0.5f * gd * (irT * irT) * r;   // C + C_q, C_q = G / (2 rho T^2)
      site_force(st[j], M, bxy.x * irT, bxy.y * irT, cc);
    }
    __syncthreads();
  } else if constexpr (MODE == MODE_INIT) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const unsigned s = rt.site(j);
      site_init(st[j], elem(in.a[0] + rb, s), elem(in.a[1] + rb, s), elem(in.a[2] + rb, s), elem(in.a[3] + rb, s));
    }
  }

  // DIRECT: xz holds the f^n of the round's six directions with v_x != 0 in pair order
  // (read once, for the transforms and the update; with the compensated state, whose collide
  // has no registers to spare, only for the transforms)
  constexpr bool DX = DIRECT && MODE == MODE_STEP;
  constexpr bool XC = DX && !COMP;
  float xz[2 * NX3][J];  // unused (and dropped by the compiler) unless DX
  // the x-derivative pairs of group k of f^n into slots 0..2, forward-transformed and
  // multiplied by i k_x / nx
  auto x_pairs = [&](int k) {
    const RowThread<NX> rt(opaque(tid));
#pragma unroll
    for (int sl = 0; sl < NX3; ++sl)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const unsigned x = rt.site(j);
#pragma unroll
        for (int h = 0; h < 2; ++h)
          xz[2 * sl + h][j] = ld_stream(P.f + (long)(1 + 8 * k + pair_dir(true, sl, h)) * P.plane + rb, x);
        lds[rt.at(sl, j)] = make_float2(xz[2 * sl][j], xz[2 * sl + 1][j]);
      }
    rows_dx_forward<NX, NX3>(lds, twx, P.kapx, tid);
  };
  if constexpr (DX) x_pairs(0);

  float m0[J], mx[J], my[J], me[J];
  // sums of the low parts of a compensated state (moments of hi + lo = moments of hi + these)
  float l0[COMP ? J : 1], lx[COMP ? J : 1], ly[COMP ? J : 1], le[COMP ? J : 1];
  // rest particle
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const unsigned s = rt.site(j);
    float fn, ln = 0.0f;
    if constexpr (MODE == MODE_STEP) {
      if constexpr (COMP) {
        const float2 hl = relax_update_comp(st[j], M, ld_stream(P.f + rb, s), ld_stream(P.flo + rb, s), feq_rest(st[j]), 0.0f,
                                            0.0f, 0.0f, force_k0(st[j], M, 0.0f));
        fn = hl.x;
        ln = hl.y;
      } else {
        fn = relax_update(st[j], M, ld_stream(P.f + rb, s), feq_rest(st[j]), 0.0f, 0.0f, 0.0f, force_k0(st[j], M, 0.0f));
      }
    } else if constexpr (MODE == MODE_INIT) {
      fn = rounded(feq_rest(st[j]));
    } else {
      fn = elem(in.a[0] + rb, s);
    }
    st_stream(P.f + rb, s, fn);
    if constexpr (COMP) {
      st_stream(P.flo + rb, s, ln);
      l0[j] = ln;
      lx[j] = ly[j] = le[j] = 0.0f;
    }
    m0[j] = fn;
    mx[j] = my[j] = me[j] = 0.0f;
  }
  if constexpr (DIRECT) {
#pragma unroll 1
    for (int rd = 0; rd < 4; ++rd) {
      const RowThread<NX> rt(opaque(tid));
      const int q0 = 1 + 8 * rd;
      // the y-parts v_y D_y f of the group: plane of direction offset d at cy + d * plane
      const float* cy = reinterpret_cast<const float*>(P.sf + (long)(q0 - 1) * hp) + rb;
      float fy[2][J];   // f^n of the two along +-y (prefetched with PREF)
      float cyv[8][J];  // y-parts by direction offset (prefetched with PREF; 0 and 4 unused)
      if constexpr (PREF) {
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int kd = 0; kd < 2; ++kd)
#pragma unroll
          for (int j = 0; j < J; ++j) fy[kd][j] = ld_stream(P.f + (long)(q0 + 2 + 4 * kd) * P.plane + rb, rt.site(j));
#pragma unroll
        for (int d = 1; d < 8; ++d) {
          if (d == 4) continue;
#pragma unroll
          for (int j = 0; j < J; ++j) cyv[d][j] = elem(cy + d * P.plane, rt.site(j));
        }
        __builtin_amdgcn_s_setprio(0);
      }
      if constexpr (MODE == MODE_STEP) {
        __syncthreads();
        rows_inverse_fft<NX, NX3>(lds, twx, tid);
      }
      const int k = rd;
      const float v2 = c_vel.v2[1 + 8 * k];
      GroupEq ge[J];
      float k0[J];
      if constexpr (MODE != MODE_SET) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
          ge[j] = group_eq(st[j], (float)group_weight((double)st[j].T, k));
          k0[j] = force_k0(st[j], M, v2);
        }
      }
      // the group's sums of f^{n+1} (and of the low parts), added to the moments once per group:
      // populations of one speed group have similar magnitudes, so this keeps the FP32
      // rounding of the moments small
      float s0[J], sx[J], sy[J], sl[COMP ? J : 1], slx[COMP ? J : 1], sly[COMP ? J : 1];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        s0[j] = sx[j] = sy[j] = 0.0f;
        if constexpr (COMP) sl[j] = slx[j] = sly[j] = 0.0f;
      }
      // u = 0..5: the six with v_x != 0 (pair u / 2, side u % 2); u = 6, 7: the two along +-y
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool xd = u < 6;
        const int d = xd ? pair_dir(true, u / 2, u % 2) : 2 + 4 * (u - 6);
        const int q = q0 + d;
        const bool hy = d != 0 && d != 4;  // has a y-part
        const float vx = c_vel.vx[q], vy = c_vel.vy[q];
        float* fQ = P.f + (long)q * P.plane + rb;
        float* lQ = COMP ? P.flo + (long)q * P.plane + rb : nullptr;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const unsigned x = rt.site(j);
          float fn, ln = 0.0f;
          if constexpr (MODE == MODE_SET) {
            fn = elem(in.a[0] + (long)q * P.plane + rb, x);
          } else {
            const float e = feq_moving(st[j], ge[j], vx, vy);
            if constexpr (MODE == MODE_STEP) {
              float c = hy ? (PREF ? cyv[d][j] : elem(cy + d * P.plane, x)) : 0.0f;
              if (xd) {
                const float2 z = lds[rt.at(u / 2, j)];
                c = fmaf(vx, u % 2 ? z.y : z.x, c);
              }
              const float f0 = xd ? (XC ? xz[xd ? u : 0][j] : ld_stream(fQ, x)) : (PREF ? fy[xd ? 0 : u - 6][j] : ld_stream(fQ, x));
              if constexpr (COMP) {
                const float2 h = relax_update_comp(st[j], M, f0, ld_stream(lQ, x), e, c, vx, vy, k0[j]);
                fn = h.x;
                ln = h.y;
              } else {
                fn = relax_update(st[j], M, f0, e, c, vx, vy, k0[j]);
              }
            } else {
              fn = rounded(e);
            }
          }
          st_stream(fQ, x, fn);
          if constexpr (COMP) {
            st_stream(lQ, x, ln);
            sl[j] += ln;
            slx[j] += vx * ln;
            sly[j] += vy * ln;
          }
          s0[j] += fn;
          sx[j] += vx * fn;
          sy[j] += vy * fn;
        }
        // without prefetch: keep one population's loads in flight at a time (bounds the live
        // registers)
        if constexpr (!PREF) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        m0[j] += s0[j];
        mx[j] += sx[j];
        my[j] += sy[j];
        me[j] += v2 * s0[j];
        if constexpr (COMP) {
          l0[j] += sl[j];
          lx[j] += slx[j];
          ly[j] += sly[j];
          le[j] += v2 * sl[j];
        }
      }
      if constexpr (DX) {
        if (rd + 1 < 4) x_pairs(rd + 1);
      }
    }
  } else {
#pragma unroll 1
    for (int rd = 0; rd < 4; ++rd) {
      const RowThread<NX> rt(opaque(tid));
      const int q0 = 1 + 8 * rd;
      float2* S = P.sf + (long)(q0 - 1) * hp;  // spectra of q0 .. q0 + 7 are consecutive planes
      PairBatchOut<NPR> io;
#pragma unroll
      for (int p = 0; p < NPR; ++p) {
        io.a[p] = S + pair_dir(DIRECT, p, 0) * hp;
        io.b[p] = S + pair_dir(DIRECT, p, 1) * hp;
        io.hb[p] = true;
      }
      float fpre[8][J];  // f^n of the round's populations (prefetched with PREF)
      if constexpr (PREF) {
        // the prefetches of a round are issued at a raised wave priority (measured faster:
        // their loads are not held up behind the transform work of the CU's other waves)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int j = 0; j < J; ++j) fpre[i][j] = ld_stream(P.f + (long)(q0 + i) * P.plane + rb, rt.site(j));
        __builtin_amdgcn_s_setprio(0);
      }
      if constexpr (MODE == MODE_STEP) {
        const PairBatch<NPR> in = conv_batch(rd);
        if constexpr (PREF) {
          rows_put_batch<NX, NPR>(lds, in, cf, tid);
          __syncthreads();
          rows_inverse_fft<NX, NPR>(lds, twx, tid);
        } else {
          rows_inverse_batch<NX, NPR>(lds, in, P.sg, twx, P.kapx, row0, tid);
        }
      }
      {
        const int k = rd;
        const float v2 = c_vel.v2[1 + 8 * k];
        GroupEq ge[J];
        float k0[J];
        if constexpr (MODE != MODE_SET) {
#pragma unroll
          for (int j = 0; j < J; ++j) {
            ge[j] = group_eq(st[j], (float)group_weight((double)st[j].T, k));
            k0[j] = force_k0(st[j], M, v2);
          }
        }
#pragma unroll
        for (int p = 0; p < NPR; ++p) {
          const int slot = p;
          const int da = pair_dir(DIRECT, p, 0), db = pair_dir(DIRECT, p, 1);
          const int qa = q0 + da, qb = q0 + db;
          const float vxa = c_vel.vx[qa], vya = c_vel.vy[qa];
          const float vxb = c_vel.vx[qb], vyb = c_vel.vy[qb];
          float* fA = P.f + (long)qa * P.plane + rb;
          float* fB = P.f + (long)qb * P.plane + rb;
          float* lA = COMP ? P.flo + (long)qa * P.plane + rb : nullptr;
          float* lB = COMP ? P.flo + (long)qb * P.plane + rb : nullptr;
#pragma unroll
          for (int j = 0; j < J; ++j) {
            const unsigned x = rt.site(j);
            const unsigned li = rt.at(slot, j);
            float fa, fb, la = 0.0f, lb = 0.0f;
            if constexpr (MODE == MODE_SET) {
              fa = elem(in.a[0] + (long)qa * P.plane + rb, x);
              fb = elem(in.a[0] + (long)qb * P.plane + rb, x);
            } else {
              const float ea = feq_moving(st[j], ge[j], vxa, vya);
              const float eb = feq_moving(st[j], ge[j], vxb, vyb);
              if constexpr (MODE == MODE_STEP) {
                const float2 c = lds[li];
                const float f0a = PREF ? fpre[da][j] : ld_stream(fA, x);
                const float f0b = PREF ? fpre[db][j] : ld_stream(fB, x);
                if constexpr (COMP) {
                  const float2 ha = relax_update_comp(st[j], M, f0a, ld_stream(lA, x), ea, c.x, vxa, vya, k0[j]);
                  const float2 hb = relax_update_comp(st[j], M, f0b, ld_stream(lB, x), eb, c.y, vxb, vyb, k0[j]);
                  fa = ha.x;
                  la = ha.y;
                  fb = hb.x;
                  lb = hb.y;
                } else {
                  fa = relax_update(st[j], M, f0a, ea, c.x, vxa, vya, k0[j]);
                  fb = relax_update(st[j], M, f0b, eb, c.y, vxb, vyb, k0[j]);
                }
              } else {
                fa = rounded(ea);
                fb = rounded(eb);
              }
            }
            st_stream(fA, x, fa);
            st_stream(fB, x, fb);
            if constexpr (COMP) {
              st_stream(lA, x, la);
              st_stream(lB, x, lb);
              l0[j] += la + lb;
              lx[j] += vxa * la + vxb * lb;
              ly[j] += vya * la + vyb * lb;
              le[j] += v2 * (la + lb);
            }
            m0[j] += fa + fb;
            mx[j] += vxa * fa + vxb * fb;
            my[j] += vya * fa + vyb * fb;
            me[j] += v2 * (fa + fb);
            lds[li] = make_float2(fa, fb);
          }
          // without prefetch: keep one pair's loads in flight at a time (bounds the live
          // registers)
          if constexpr (!PREF) __builtin_amdgcn_sched_barrier(0);
        }
      }
      if constexpr (PREF) {
        __builtin_amdgcn_s_setprio(1);
        if (rd + 1 < 4) cf = rows_fetch_batch<NX, NPR>(conv_batch(rd + 1), P.sg, P.kapx, row0, tid);
        __builtin_amdgcn_s_setprio(0);
      }
      rows_forward_batch<NX, NPR>(lds, io, P.sg, twx, row0, tid);
    }
  }
  // moments of the new state and their row spectra
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if constexpr (COMP) {
      m0[j] += l0[j];
      mx[j] += lx[j];
      my[j] += ly[j];
      me[j] += le[j];
    }
    const unsigned s = rt.site(j);
    const float r = m0[j];
    const float ir = 1.0f / r;
    const float ux = mx[j] * ir, uy = my[j] * ir;
    const float T = 0.5f * me[j] * ir - 0.5f * (ux * ux + uy * uy);
    elem(mac, s) = r;
    elem(mac + P.plane, s) = ux;
    elem(mac + 2 * P.plane, s) = uy;
    elem(mac + 3 * P.plane, s) = T;
    lds[rt.at(0, j)] = make_float2(r, ux);
    lds[rt.at(1, j)] = make_float2(uy, T);
  }
  PairBatchOut<2> mo{{P.sm, P.sm + 2 * hp}, {P.sm + hp, P.sm + 3 * hp}, {true, true}};
  rows_forward_batch<NX, 2>(lds, mo, P.sg, twx, row0, tid);
}

template <int NX, int MODE, bool COMP, bool XCOL = false>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_collide(RowArgs A, Inputs in) {
  const int s = blockIdx.y;
  if (retired(A.state, A.id[s])) return;
  assume_planes(A.P[s]);
  rows_collide<NX, MODE, COMP, XCOL>(A.P[s], A.M[s], in, blockIdx.x);
}

// Residual pass, step 1: momentum j = rho u of the current state and its row spectra
// (into stage-1 spectral planes 0 and 1, free between steps).
template <int NX>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_momentum(RowArgs A) {
  const int slot = blockIdx.y;
  if (retired(A.state, A.id[slot])) return;
  extern __shared__ float2 lds[];
  const Planes& P = A.P[slot];
  assume_planes(P);
  const int tid = threadIdx.x;
  const RowThread<NX> rt(tid);
  const float* mac = P.macro + (long)blockIdx.x * RowGeom<NX>::RB * NX;
  const long hp = P.plane / 2;
  const float2* twx = row_twiddles<NX>(lds, P.twx, tid);
#pragma unroll
  for (int j = 0; j < RowGeom<NX>::J; ++j) {
    const unsigned s = rt.site(j);
    const float r = elem(mac, s);
    lds[rt.at(0, j)] = make_float2(r * elem(mac + P.plane, s), r * elem(mac + 2 * P.plane, s));
  }
  PairBatchOut<1> o{{P.s1}, {P.s1 + hp}, {true}};
  rows_forward_batch<NX, 1>(lds, o, P.sg, twx, blockIdx.x * RowGeom<NX>::RB, tid);
}

// Residual pass, step 3 (after the column pass has formed the spectrum of D.j in stage-1
// plane 2): inverse row transform, block max |dt D.j| and a non-finite flag into the
// partials read by the global reduction and the batch poll.  In exact arithmetic D.j is the
// sum over populations of the convection terms (the transforms are linear), so dt max|D.j|
// is the density change of the next step; formed from j it carries FP32 rounding of j, not
// of the 33 much larger population terms.
template <int NX>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_residual(RowArgs A) {
  const int slot = blockIdx.y;
  if (retired(A.state, A.id[slot])) return;
  extern __shared__ float2 lds[];
  const Planes& P = A.P[slot];
  assume_planes(P);
  const int tid = threadIdx.x;
  const RowThread<NX> rt(tid);
  const long hp = P.plane / 2;
  const float2* twx = row_twiddles<NX>(lds, P.twx, tid);
  PairBatch<1> b1 = empty_batch<1>();
  set_term(b1, 0, 0, 0, P.s1 + 2 * hp, 1.0f, TERM_ONE);
  rows_inverse_batch<NX, 1>(lds, b1, P.sg, twx, P.kapx, blockIdx.x * RowGeom<NX>::RB, tid);
  float m = 0.0f;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < RowGeom<NX>::J; ++j) {
    const float v = lds[rt.at(0, j)].x;
    m = fmaxf(m, fabsf(v));
    bad |= nonfinite(v);
  }
  __shared__ float red[16][2];
  const int wave = tid / 64, lane = tid % 64;
  m = wave_max(m);
  const float badf = wave_max(bad ? 1.0f : 0.0f);
  if (lane == 0) {
    red[wave][0] = m;
    red[wave][1] = badf;
  }
  __syncthreads();
  if (tid == 0) {
    constexpr int NW = (RowGeom<NX>::NT + 63) / 64;
    float a = 0.0f, bd = 0.0f;
    for (int w = 0; w < NW; ++w) {
      a = fmaxf(a, red[w][0]);
      bd = fmaxf(bd, red[w][1]);
    }
    P.part_f[2 * blockIdx.x] = a;
    P.part_f[2 * blockIdx.x + 1] = bd;
  }
}

// Real plane(s) -> packed row spectra (b may be null).
template <int NX>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_forward_real(const float* __restrict__ a,
                                                                       const float* __restrict__ b,
                                                                       float2* sa, float2* sb, SpecGeom sg,
                                                                       const float2* twx, int nx) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const RowThread<NX> rt(tid);
  const long rb = (long)blockIdx.x * RowGeom<NX>::RB * NX;
#pragma unroll
  for (int j = 0; j < RowGeom<NX>::J; ++j) {
    const unsigned s = rt.site(j);
    lds[rt.at(0, j)] = make_float2(elem(a + rb, s), b ? elem(b + rb, s) : 0.0f);
  }
  twx = row_twiddles<NX>(lds, twx, tid);
  PairBatchOut<1> o{{sa}, {sb}, {sb != nullptr}};
  rows_forward_batch<NX, 1>(lds, o, sg, twx, blockIdx.x * RowGeom<NX>::RB, tid);
}

// The 32 real convection planes of the flux-limiter scheme -> the population spectra (packed row
// spectra, plane pair p -> spectra 2p and 2p + 1), for up to kSchemeSlots instances of one grid
// size: blockIdx.y = pair, blockIdx.z = slot.
struct PlaneFwdInst {
  const float* src;        // [32][ny][nx]
  float2* dst;             // [32] population spectra
  const float2* twx;       // row twiddles
  SpecGeom sg;
  long plane;              // nx * ny
  int id;
};

struct PlaneFwdArgs {
  PlaneFwdInst c[kSchemeSlots];
  const int* state;
};

template <int NX>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_forward_planes(PlaneFwdArgs A) {
  const PlaneFwdInst& I = A.c[blockIdx.z];
  if (retired(A.state, I.id)) return;
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const RowThread<NX> rt(tid);
  const long rb = (long)blockIdx.x * RowGeom<NX>::RB * NX;
  const long p2 = 2 * (long)blockIdx.y;
  const float* a = I.src + p2 * I.plane;
  const float* b = a + I.plane;
#pragma unroll
  for (int j = 0; j < RowGeom<NX>::J; ++j) {
    const unsigned s = rt.site(j);
    lds[rt.at(0, j)] = make_float2(elem(a + rb, s), elem(b + rb, s));
  }
  const float2* twx = row_twiddles<NX>(lds, I.twx, tid);
  const long hp = I.plane / 2;
  PairBatchOut<1> o{{I.dst + p2 * hp}, {I.dst + (p2 + 1) * hp}, {true}};
  rows_forward_batch<NX, 1>(lds, o, I.sg, twx, blockIdx.x * RowGeom<NX>::RB, tid);
}

// Packed row spectra -> real plane(s) (b may be null).
template <int NX>
__global__ __launch_bounds__(RowGeom<NX>::NT) void k_rows_inverse_real(const float2* sa, const float2* sb,
                                                                       float* __restrict__ a, float* __restrict__ b,
                                                                       SpecGeom sg, const float2* twx,
                                                                       const float* __restrict__ kapx, int nx) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const RowThread<NX> rt(tid);
  const long rb = (long)blockIdx.x * RowGeom<NX>::RB * NX;
  const float2* a1[1] = {sa};
  twx = row_twiddles<NX>(lds, twx, tid);
  const float2* b1[1] = {sb};
  rows_inverse_batch<NX, 1>(lds, plain_batch<1>(a1, b1), sg, twx, kapx, blockIdx.x * RowGeom<NX>::RB, tid);
#pragma unroll
  for (int j = 0; j < RowGeom<NX>::J; ++j) {
    const unsigned s = rt.site(j);
    const float2 v = lds[rt.at(0, j)];
    elem(a + rb, s) = v.x;
    if (b) elem(b + rb, s) = v.y;
  }
}

}  // namespace fftlb
