// C ABI of the FFT-LB solver: argument checking, workspace layout, tables, kernel
// dispatch over grid sizes, and HIP-graph capture of the time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "fftlb.h"
#include "kernels.hpp"

using namespace fftlb;

namespace {

thread_local char g_last_error[512] = "";

void set_error(const char* what, hipError_t e) {
  std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(call)                                        \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) {                                  \
      set_error(#call, e_);                                  \
      return FFTLB_EHIP;                                     \
    }                                                        \
  } while (0)

constexpr int kMaxN = 2048;

// Grid sizes with compiled kernels: powers of two, and 3 * 2^p from 48 to 768.
bool size_supported(int n) { return is_pow2(n) || (n % 3 == 0 && is_pow2(n / 3) && n >= 48 && n <= 768); }

int floor_pow2(int n) { return n < 1 ? 0 : 1 << ilog2(n); }
constexpr int kStepsPerGraph = 16;

int row_rows_per_block(int nx) {
  const int tpr = nx / (nx >= 2048 ? 4 : 2);  // threads per row, as in RowGeom
  return tpr >= 64 ? 1 : 64 / tpr;
}

// Spectral tile width: the largest power of two <= 16 that divides nx/2.
int tile_width(int nx) { return std::min(16, (nx / 2) & -(nx / 2)); }

// Columns per block of the column kernels (a power of two dividing the tile width): the LDS
// block is ny * cw * 8 bytes per buffer, kept within 64 KB (1 buffer for the convection
// pass, up to 4 for the derivative groups).
int conv_cols(int ny, int tw) { return std::min(tw, floor_pow2(std::max(1, std::min(16, 8192 / ny)))); }
int multi_cols(int ny, int tw) { return std::min(tw, floor_pow2(std::max(1, std::min(16, 2048 / ny)))); }

bool config_ok(const fftlb_config* c) {
  if (!c) return false;
  if (!size_supported(c->nx) || !size_supported(c->ny)) return false;
  if (c->nx < 8 || c->nx > kMaxN || c->ny < 4 || c->ny > kMaxN) return false;
  if (c->ny % row_rows_per_block(c->nx)) return false;
  auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
  auto nonneg = [](double v) { return std::isfinite(v) && v >= 0.0; };
  if (!pos(c->dx) || !pos(c->dy) || !pos(c->dt)) return false;
  if (!(c->tau > 0.0) || std::isnan(c->tau)) return false;
  if (!nonneg(c->K) || !nonneg(c->H) || !nonneg(c->a) || !nonneg(c->b)) return false;
  if (!std::isfinite(c->zeta) || !std::isfinite(c->q)) return false;
  if (c->filter_order < 0 || c->filter_order > 4) return false;
  if (c->reserved != 0) return false;
  return true;
}

struct Layout {
  size_t f, sf, sm, s1, s2i, s2o, macro, cpl, twx, twy, kx, ky, pd, pf, total;
};

size_t align_up(size_t v) { return (v + FFTLB_WORKSPACE_ALIGN - 1) / FFTLB_WORKSPACE_ALIGN * FFTLB_WORKSPACE_ALIGN; }

Layout make_layout(int nx, int ny) {
  const size_t plane = (size_t)nx * ny * sizeof(float);  // a real plane, or a half-spectrum plane
  const size_t nblk = (size_t)ny / row_rows_per_block(nx);
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.f = take(33 * plane);
  L.sf = take(32 * plane);
  L.sm = take(4 * plane);
  L.s1 = take(6 * plane);
  L.s2i = take(5 * plane);
  L.s2o = take(3 * plane);
  L.macro = take(4 * plane);
  L.cpl = take(plane);
  L.twx = take((size_t)nx * sizeof(float2));
  L.twy = take((size_t)ny * sizeof(float2));
  L.kx = take((size_t)(nx / 2) * sizeof(float));
  L.ky = take((size_t)ny * sizeof(float));
  L.pd = take(nblk * 6 * sizeof(double));
  L.pf = take(nblk * 2 * sizeof(float));
  L.total = o;
  return L;
}

// Windowed wavenumber k_m (Eqs. (44)-(47)) of signed index n on a grid of N points with
// spacing d; the Nyquist index -N/2 gets 0.  m = 0 is the exact wavenumber.
double windowed_k(int n, int N, double d, int m) {
  if (2 * n == -N || 2 * n == N) return 0.0;
  const double k = 2.0 * M_PI * n / (N * d);
  if (m == 0) return k;
  static const double c[4] = {1.0, 1.0 / 6.0, 3.0 / 40.0, 5.0 / 112.0};
  const double s = std::sin(M_PI * (double)n / N);
  double acc = 0.0, sp = s;
  for (int j = 0; j < m; ++j) {
    acc += c[j] * sp;
    sp *= s * s;
  }
  return 2.0 / d * acc;
}

}  // namespace

struct fftlb_handle {
  fftlb_config cfg;
  int device;
  int nx, ny, tw;
  Layout L;
  Planes P;
  Model M;
  float2* twy;
  float* kapx;
  float* kapy;
  int nblk_rows;
  int64_t steps;
  hipStream_t cap, cap2;   // capture streams (the second carries the concurrent branch)
  hipEvent_t fork, join;
  hipGraphExec_t g1, gN;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------------------------------
// Kernel dispatch over compile-time sizes
// ---------------------------------------------------------------------------

template <template <int> class F, typename... A>
int dispatch_nx(int nx, A&&... a) {
  switch (nx) {
    case 8: return F<8>::run(a...);
    case 16: return F<16>::run(a...);
    case 48: return F<48>::run(a...);
    case 96: return F<96>::run(a...);
    case 192: return F<192>::run(a...);
    case 384: return F<384>::run(a...);
    case 768: return F<768>::run(a...);
    case 32: return F<32>::run(a...);
    case 64: return F<64>::run(a...);
    case 128: return F<128>::run(a...);
    case 256: return F<256>::run(a...);
    case 512: return F<512>::run(a...);
    case 1024: return F<1024>::run(a...);
    case 2048: return F<2048>::run(a...);
  }
  return FFTLB_EINVAL;
}

// radix-16 passes: one 16-point butterfly per thread per pass
constexpr int col_threads(int ny, int cw) { return std::min(1024, std::max(64, ny * cw / 16)); }

template <int NY, int CW>
struct ColConv {
  static int run(hipStream_t s, fftlb_handle* h) {
    if constexpr (NY * CW > 8192) {
      return FFTLB_EINVAL;
    } else {
      constexpr int NT = col_threads(NY, CW);
      const int nblocks = 24 * ((h->nx / 2) / CW);   // 24 populations with v_y != 0
      hipLaunchKernelGGL((k_col_conv<NY, CW, NT>), dim3(nblocks), dim3(NT), lds_alloc(NY * CW) * sizeof(float2), s,
                         h->P.sf, h->twy, h->kapx, h->kapy, h->nx, h->tw, h->M.scale);
      return FFTLB_OK;
    }
  }
};

template <int NY, int CW>
struct ColMulti {
  static int run(hipStream_t s, fftlb_handle* h, const ColLaunch& L, int ngroups, int maxin) {
    if constexpr (NY * CW * 4 > 8192) {
      return FFTLB_EINVAL;
    } else {
      constexpr int NT = col_threads(NY, CW);
      const int nsub = (h->nx / 2) / CW;
      (void)maxin;  // the work block sits after room for three inputs
      const size_t lds = (size_t)lds_alloc(4 * NY * CW) * sizeof(float2);
      hipLaunchKernelGGL((k_col_multi<NY, CW, NT>), dim3(nsub, ngroups), dim3(NT), lds, s, L, h->twy, h->kapx,
                         h->kapy, h->nx, h->tw, h->M.scale);
      return FFTLB_OK;
    }
  }
};

template <template <int, int> class F, int NY, typename... A>
int dispatch_cw(int cw, A&&... a) {
  switch (cw) {
    case 1: return F<NY, 1>::run(a...);
    case 2: return F<NY, 2>::run(a...);
    case 4: return F<NY, 4>::run(a...);
    case 8: return F<NY, 8>::run(a...);
    case 16: return F<NY, 16>::run(a...);
  }
  return FFTLB_EINVAL;
}

template <template <int, int> class F, typename... A>
int dispatch_ny(int ny, int cw, A&&... a) {
  switch (ny) {
    case 4: return dispatch_cw<F, 4>(cw, a...);
    case 8: return dispatch_cw<F, 8>(cw, a...);
    case 16: return dispatch_cw<F, 16>(cw, a...);
    case 48: return dispatch_cw<F, 48>(cw, a...);
    case 96: return dispatch_cw<F, 96>(cw, a...);
    case 192: return dispatch_cw<F, 192>(cw, a...);
    case 384: return dispatch_cw<F, 384>(cw, a...);
    case 768: return dispatch_cw<F, 768>(cw, a...);
    case 32: return dispatch_cw<F, 32>(cw, a...);
    case 64: return dispatch_cw<F, 64>(cw, a...);
    case 128: return dispatch_cw<F, 128>(cw, a...);
    case 256: return dispatch_cw<F, 256>(cw, a...);
    case 512: return dispatch_cw<F, 512>(cw, a...);
    case 1024: return dispatch_cw<F, 1024>(cw, a...);
    case 2048: return dispatch_cw<F, 2048>(cw, a...);
  }
  return FFTLB_EINVAL;
}

template <int NX>
struct RowStage2 {
  static int run(hipStream_t s, fftlb_handle* h) {
    hipLaunchKernelGGL(k_rows_stage2<NX>, dim3(h->nblk_rows), dim3(RowGeom<NX>::NT),
                       RowGeom<NX>::LDS * sizeof(float2), s, h->P, h->M);
    return FFTLB_OK;
  }
};

template <int MODE>
struct RowCollideMode {
  template <int NX>
  struct K {
    static int run(hipStream_t s, fftlb_handle* h, const Planes& P) {
      hipLaunchKernelGGL((k_rows_collide<NX, MODE>), dim3(h->nblk_rows), dim3(RowGeom<NX>::NT),
                         RowGeom<NX>::LDS * sizeof(float2), s, P, h->M);
      return FFTLB_OK;
    }
  };
};

template <int NX>
struct RowFwdReal {
  static int run(hipStream_t s, fftlb_handle* h, const float* a, const float* b, float2* sa, float2* sb) {
    hipLaunchKernelGGL(k_rows_forward_real<NX>, dim3(h->nblk_rows), dim3(RowGeom<NX>::NT),
                       RowGeom<NX>::LDS * sizeof(float2), s, a, b, sa, sb, h->P.sg, h->P.twx, h->nx);
    return FFTLB_OK;
  }
};

template <int NX>
struct RowInvReal {
  static int run(hipStream_t s, fftlb_handle* h, const float2* sa, const float2* sb, float* a, float* b) {
    hipLaunchKernelGGL(k_rows_inverse_real<NX>, dim3(h->nblk_rows), dim3(RowGeom<NX>::NT),
                       RowGeom<NX>::LDS * sizeof(float2), s, sa, sb, a, b, h->P.sg, h->P.twx, h->P.kapx, h->nx);
    return FFTLB_OK;
  }
};

// ---------------------------------------------------------------------------
// Step building blocks
// ---------------------------------------------------------------------------

ColGroup group(std::initializer_list<const float2*> in, std::initializer_list<float2*> out,
               std::initializer_list<std::initializer_list<int>> kinds) {
  ColGroup g{};
  g.nin = (int)in.size();
  g.nout = (int)out.size();
  int i = 0;
  for (auto p : in) g.in[i++] = p;
  i = 0;
  for (auto p : out) g.out[i++] = p;
  i = 0;
  for (auto& row : kinds) {
    int j = 0;
    for (int k : row) g.kind[i][j++] = k;
    ++i;
  }
  return g;
}

int launch_stage1(fftlb_handle* h, hipStream_t s) {
  const long hp = (long)h->nx * h->ny / 2;
  float2* sm = h->P.sm;
  float2* s1 = h->P.s1;
  ColLaunch L{};
  // Only the y-derivatives need the column pass; x-derivatives are formed in the stage-2
  // row kernel from the moment spectra.  s1 = [D_y rho, D_yy rho, D_y ux, D_y uy, D_y theta, D_y T]
  // rho -> D_y rho, D_yy rho
  L.g[0] = group({sm}, {s1, s1 + hp}, {{MK_IKY}, {MK_KYY}});
  // ux, uy -> D_y ux, D_y uy, D_y theta = D_y D_x ux + D_yy uy
  L.g[1] = group({sm + hp, sm + 2 * hp}, {s1 + 2 * hp, s1 + 3 * hp, s1 + 4 * hp},
                 {{MK_IKY, MK_NONE}, {MK_NONE, MK_IKY}, {MK_KXY, MK_KYY}});
  // T -> D_y T
  L.g[2] = group({sm + 3 * hp}, {s1 + 5 * hp}, {{MK_IKY}});
  return dispatch_ny<ColMulti>(h->ny, multi_cols(h->ny, h->tw), s, h, L, 3, 2);
}

int launch_stage2_cols(fftlb_handle* h, hipStream_t s) {
  const long hp = (long)h->nx * h->ny / 2;
  float2* i2 = h->P.s2i;
  float2* o2 = h->P.s2o;
  ColLaunch L{};
  // B^x = D_x(S + Lxx) + D_y Lxy,  B^y = D_x Lxy + D_y(S + Lyy)
  L.g[0] = group({i2, i2 + hp, i2 + 2 * hp}, {o2, o2 + hp},
                 {{MK_IKX, MK_IKY, MK_NONE}, {MK_NONE, MK_IKX, MK_IKY}});
  // G = D_x gx + D_y gy
  L.g[1] = group({i2 + 3 * hp, i2 + 4 * hp}, {o2 + 2 * hp}, {{MK_IKX, MK_IKY}});
  return dispatch_ny<ColMulti>(h->ny, multi_cols(h->ny, h->tw), s, h, L, 2, 3);
}

constexpr int kNumStages = 5;

// One kernel of the step: 0 convection columns, 1 stage-1 columns, 2 stage-2 rows,
// 3 stage-2 columns, 4 collide rows.
int enqueue_stage(fftlb_handle* h, int stage, hipStream_t s) {
  switch (stage) {
    case 0: return dispatch_ny<ColConv>(h->ny, conv_cols(h->ny, h->tw), s, h);
    case 1: return launch_stage1(h, s);
    case 2: return dispatch_nx<RowStage2>(h->nx, s, h);
    case 3: return launch_stage2_cols(h, s);
    case 4: return dispatch_nx<RowCollideMode<MODE_STEP>::K>(h->nx, s, h, h->P);
  }
  return FFTLB_EINVAL;
}

int enqueue_step(fftlb_handle* h, hipStream_t s) {
  for (int k = 0; k < kNumStages; ++k) {
    const int rc = enqueue_stage(h, k, s);
    if (rc) return rc;
  }
  return FFTLB_OK;
}

// The step as captured into a graph: the convection column pass (stage 0) runs on a
// second branch, concurrently with the force pipeline (stages 1-3); the collide
// (stage 4) joins both.
int enqueue_step_forked(fftlb_handle* h, hipStream_t s) {
  int rc;
  HIP_TRY(hipEventRecord(h->fork, s));
  HIP_TRY(hipStreamWaitEvent(h->cap2, h->fork, 0));
  if ((rc = enqueue_stage(h, 0, h->cap2))) return rc;
  HIP_TRY(hipEventRecord(h->join, h->cap2));
  for (int k = 1; k <= 3; ++k)
    if ((rc = enqueue_stage(h, k, s))) return rc;
  HIP_TRY(hipStreamWaitEvent(s, h->join, 0));
  return enqueue_stage(h, 4, s);
}

int capture(fftlb_handle* h, int nsteps, hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
  int rc = FFTLB_OK;
  for (int i = 0; i < nsteps && rc == FFTLB_OK; ++i) rc = enqueue_step_forked(h, h->cap);
  hipError_t le = hipGetLastError();
  hipError_t ee = hipStreamEndCapture(h->cap, &graph);
  if (rc != FFTLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (le != hipSuccess) {
    set_error("kernel launch during capture", le);
    if (graph) (void)hipGraphDestroy(graph);
    return FFTLB_EHIP;
  }
  if (ee != hipSuccess) {
    set_error("hipStreamEndCapture", ee);
    return FFTLB_EHIP;
  }
  hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    set_error("hipGraphInstantiate", ie);
    return FFTLB_EHIP;
  }
  return FFTLB_OK;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(what, e);
    return FFTLB_EHIP;
  }
  return FFTLB_OK;
}

}  // namespace

extern "C" {

int fftlb_workspace_bytes(const fftlb_config* cfg, size_t* bytes) {
  if (!config_ok(cfg) || !bytes) return FFTLB_EINVAL;
  *bytes = make_layout(cfg->nx, cfg->ny).total;
  return FFTLB_OK;
}

int fftlb_init(const fftlb_config* cfg, void* workspace, size_t ws_bytes, const float* rho0, const float* ux0,
               const float* uy0, const float* T0, void* stream, fftlb_handle** out) {
  if (!out) return FFTLB_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg) || !rho0 || !ux0 || !uy0 || !T0) return FFTLB_EINVAL;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % FFTLB_WORKSPACE_ALIGN)) return FFTLB_ENOSPC;
  const Layout L = make_layout(cfg->nx, cfg->ny);
  if (ws_bytes < L.total) return FFTLB_ENOSPC;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  fftlb_handle* h = new (std::nothrow) fftlb_handle();
  if (!h) return FFTLB_EINVAL;
  h->cfg = *cfg;
  h->nx = cfg->nx;
  h->ny = cfg->ny;
  h->tw = tile_width(cfg->nx);
  h->L = L;
  h->steps = 0;
  h->g1 = h->gN = nullptr;
  h->cap = h->cap2 = nullptr;
  h->fork = h->join = nullptr;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return FFTLB_EHIP;
  }
  char* ws = static_cast<char*>(workspace);
  Planes& P = h->P;
  P.f = reinterpret_cast<float*>(ws + L.f);
  P.sf = reinterpret_cast<float2*>(ws + L.sf);
  P.sm = reinterpret_cast<float2*>(ws + L.sm);
  P.s1 = reinterpret_cast<float2*>(ws + L.s1);
  P.s2i = reinterpret_cast<float2*>(ws + L.s2i);
  P.s2o = reinterpret_cast<float2*>(ws + L.s2o);
  P.macro = reinterpret_cast<float*>(ws + L.macro);
  P.cpl = reinterpret_cast<float*>(ws + L.cpl);
  P.twx = reinterpret_cast<const float2*>(ws + L.twx);
  P.kapx = reinterpret_cast<const float*>(ws + L.kx);
  P.part_d = reinterpret_cast<double*>(ws + L.pd);
  P.part_f = reinterpret_cast<float*>(ws + L.pf);
  P.in0 = P.in1 = P.in2 = P.in3 = nullptr;
  P.nx = h->nx;
  P.ny = h->ny;
  P.plane = (long)h->nx * h->ny;
  P.sg.ny = h->ny;
  P.sg.tw = h->tw;
  P.sg.log2tw = ilog2(h->tw);
  h->twy = reinterpret_cast<float2*>(ws + L.twy);
  h->kapx = reinterpret_cast<float*>(ws + L.kx);
  h->kapy = reinterpret_cast<float*>(ws + L.ky);
  h->nblk_rows = h->ny / row_rows_per_block(h->nx);

  Model& M = h->M;
  M.dt = (float)cfg->dt;
  M.omega = std::isinf(cfg->tau) ? 0.0f : (float)(cfg->dt / cfg->tau);
  M.K = (float)cfg->K;
  M.H = (float)cfg->H;
  M.zeta = (float)cfg->zeta;
  M.q = (float)cfg->q;
  M.a = (float)cfg->a;
  M.b = (float)cfg->b;
  M.scale = (float)(1.0 / ((double)h->nx * h->ny));

  // Twiddles exp(-2 pi i j/N) and windowed wavenumbers, in FP64, stored FP32.
  std::vector<float2> twx(h->nx), twy(h->ny);
  for (int j = 0; j < h->nx; ++j)
    twx[j] = make_float2((float)std::cos(2.0 * M_PI * j / h->nx), (float)-std::sin(2.0 * M_PI * j / h->nx));
  for (int j = 0; j < h->ny; ++j)
    twy[j] = make_float2((float)std::cos(2.0 * M_PI * j / h->ny), (float)-std::sin(2.0 * M_PI * j / h->ny));
  std::vector<float> kx(h->nx / 2), ky(h->ny);
  for (int k = 0; k < h->nx / 2; ++k) kx[k] = (float)windowed_k(k, h->nx, cfg->dx, cfg->filter_order);
  for (int k = 0; k < h->ny; ++k)
    ky[k] = (float)windowed_k(k < h->ny / 2 ? k : k - h->ny, h->ny, cfg->dy, cfg->filter_order);

  int rc = FFTLB_OK;
  {
    DeviceGuard dg(h->device);
    auto fail = [&](int code) {
      if (h->cap) (void)hipStreamDestroy(h->cap);
      if (h->cap2) (void)hipStreamDestroy(h->cap2);
      if (h->fork) (void)hipEventDestroy(h->fork);
      if (h->join) (void)hipEventDestroy(h->join);
      delete h;
      return code;
    };
    // default-priority streams; events without timing
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&h->cap2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->join, hipEventDisableTiming) != hipSuccess) {
      set_error("stream/event creation", hipErrorUnknown);
      return fail(FFTLB_EHIP);
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(ws + L.twx, twx.data(), twx.size() * sizeof(float2), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.twy, twy.data(), twy.size() * sizeof(float2), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.kx, kx.data(), kx.size() * sizeof(float), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.ky, ky.data(), ky.size() * sizeof(float), hipMemcpyHostToDevice, s))) {
      set_error("table upload", e);
      return fail(FFTLB_EHIP);
    }
    Planes Pi = P;
    Pi.in0 = rho0;
    Pi.in1 = ux0;
    Pi.in2 = uy0;
    Pi.in3 = T0;
    rc = dispatch_nx<RowCollideMode<MODE_INIT>::K>(h->nx, s, h, Pi);
    if (rc == FFTLB_OK) rc = check_launch("init kernel");
    if (rc == FFTLB_OK && (e = hipStreamSynchronize(s)) != hipSuccess) {
      set_error("hipStreamSynchronize", e);
      rc = FFTLB_EHIP;
    }
    if (rc != FFTLB_OK) return fail(rc);
  }
  *out = h;
  return FFTLB_OK;
}

int fftlb_step(fftlb_handle* h, int64_t nsteps, void* stream) {
  if (!h || nsteps < 0) return FFTLB_EINVAL;
  if (nsteps == 0) return FFTLB_OK;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc;
  if (!h->g1 && (rc = capture(h, 1, &h->g1))) return rc;
  if (nsteps >= kStepsPerGraph && !h->gN && (rc = capture(h, kStepsPerGraph, &h->gN))) return rc;
  int64_t left = nsteps;
  while (left >= kStepsPerGraph) {
    HIP_TRY(hipGraphLaunch(h->gN, s));
    left -= kStepsPerGraph;
  }
  while (left > 0) {
    HIP_TRY(hipGraphLaunch(h->g1, s));
    --left;
  }
  h->steps += nsteps;
  return FFTLB_OK;
}

int fftlb_run_stage(fftlb_handle* h, int32_t stage, int32_t reps, void* stream) {
  if (!h || stage < 0 || stage >= kNumStages || reps < 0) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < reps; ++i) {
    const int rc = enqueue_stage(h, stage, s);
    if (rc) return rc;
  }
  if (stage == kNumStages - 1) h->steps += reps;
  return check_launch("run_stage");
}

int fftlb_moments(fftlb_handle* h, float* rho, float* ux, float* uy, float* T, double* globals, void* stream) {
  if (!h) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t pb = (size_t)h->nx * h->ny * sizeof(float);
  float* outs[4] = {rho, ux, uy, T};
  for (int i = 0; i < 4; ++i)
    if (outs[i]) HIP_TRY(hipMemcpyAsync(outs[i], h->P.macro + (size_t)i * h->nx * h->ny, pb,
                                        hipMemcpyDeviceToDevice, s));
  if (globals) {
    int rc;
    if ((rc = launch_stage1(h, s))) return rc;
    if ((rc = dispatch_nx<RowStage2>(h->nx, s, h))) return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, h->P.part_d, h->nblk_rows, h->P.part_f,
                       h->nblk_rows, h->steps > 0 ? 1 : 0, h->cfg.dx * h->cfg.dy, h->cfg.dt, (double)h->steps,
                       globals);
    if ((rc = check_launch("moments"))) return rc;
  }
  return FFTLB_OK;
}

int fftlb_get_state(fftlb_handle* h, float* f, void* stream) {
  if (!h || !f) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  HIP_TRY(hipMemcpyAsync(f, h->P.f, (size_t)33 * h->nx * h->ny * sizeof(float), hipMemcpyDeviceToDevice,
                         reinterpret_cast<hipStream_t>(stream)));
  return FFTLB_OK;
}

int fftlb_set_state(fftlb_handle* h, const float* f, void* stream) {
  if (!h || !f) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  Planes Ps = h->P;
  Ps.in0 = f;
  int rc = dispatch_nx<RowCollideMode<MODE_SET>::K>(h->nx, reinterpret_cast<hipStream_t>(stream), h, Ps);
  if (rc == FFTLB_OK) rc = check_launch("set_state");
  return rc;
}

int fftlb_derivative(fftlb_handle* h, const float* g, float* out, int32_t op, void* stream) {
  if (!h || !g || !out || g == out || op < 0 || op > 2) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float2* src = h->P.s1;
  float2* dst = h->P.s1 + (long)h->nx * h->ny / 2;
  int rc;
  if ((rc = dispatch_nx<RowFwdReal>(h->nx, s, h, g, (const float*)nullptr, src, (float2*)nullptr))) return rc;
  ColLaunch L{};
  // the derivative entry point runs every operator through the full 2D pass
  const int kind = op == 0 ? MK_IKX : (op == 1 ? MK_IKY : MK_LAP);
  L.g[0] = group({src}, {dst}, {{kind}});
  if ((rc = dispatch_ny<ColMulti>(h->ny, multi_cols(h->ny, h->tw), s, h, L, 1, 1))) return rc;
  if ((rc = dispatch_nx<RowInvReal>(h->nx, s, h, (const float2*)dst, (const float2*)nullptr, out, (float*)nullptr)))
    return rc;
  return check_launch("derivative");
}

int fftlb_destroy(fftlb_handle* h) {
  if (!h) return FFTLB_EINVAL;
  {
    DeviceGuard dg(h->device);
    // graphs may still be running on the caller's streams
    (void)hipDeviceSynchronize();
    if (h->g1) (void)hipGraphExecDestroy(h->g1);
    if (h->gN) (void)hipGraphExecDestroy(h->gN);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->cap2) (void)hipStreamDestroy(h->cap2);
    if (h->fork) (void)hipEventDestroy(h->fork);
    if (h->join) (void)hipEventDestroy(h->join);
  }
  delete h;
  return FFTLB_OK;
}

const char* fftlb_strerror(int code) {
  switch (code) {
    case FFTLB_OK: return "ok";
    case FFTLB_EINVAL: return "invalid argument or unsupported configuration";
    case FFTLB_ENOSPC: return "workspace too small or misaligned";
    case FFTLB_EHIP: return "HIP runtime error";
    case FFTLB_EUNSTABLE: return "non-finite values in the state";
  }
  return "unknown error";
}

const char* fftlb_last_error(void) { return g_last_error; }

}  // extern "C"
