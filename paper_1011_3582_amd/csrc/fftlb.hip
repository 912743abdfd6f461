// C ABI of the FFT-LB solver: argument checking, workspace layout, tables, kernel
// dispatch over grid sizes, HIP-graph capture of the time step, column-plan autotuning
// and batches of instances of uneven grid sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "fftlb.h"
#include "launch.hpp"
#include "reduce.hpp"
#include "stencil.hpp"

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

#define RC_TRY(call)          \
  do {                        \
    const int rc_ = (call);   \
    if (rc_) return rc_;      \
  } while (0)

constexpr int kMaxN = 2048;
// Step graphs of 1, 2, 4, ..., 2^(kGraphLevels - 1) steps: a call of n steps replays the
// largest one floor(n / 16) times and the rest as its binary digits (at most four more
// launches), so no count of steps falls back to one replay per step.
constexpr int kGraphLevels = 5;
constexpr int kStepsPerGraph = 1 << (kGraphLevels - 1);
constexpr int kMaxPollEvery = 1000;

// Grid sizes with compiled kernels: powers of two, and 3 * 2^p from 48 to 768.
bool size_supported(int n) { return is_pow2(n) || (n % 3 == 0 && is_pow2(n / 3) && n >= 48 && n <= 768); }

int floor_pow2(int n) { return n < 1 ? 0 : 1 << ilog2(n); }

int row_rows_per_block(int nx) {
  const int tpr = nx / (nx >= 2048 ? 4 : 2);  // threads per row, as in RowGeom
  return tpr >= 64 ? 1 : 64 / tpr;
}

// Spectral tile width: the largest power of two <= 16 that divides nx/2.
int tile_width(int nx) { return std::min(16, (nx / 2) & -(nx / 2)); }

// Largest column counts per block the LDS budget allows: one buffer of ny * cw float2 for the
// convection pass, kMultiSlots for the derivative passes (their largest group).
int conv_cols_max(int ny, int tw) { return std::min(tw, floor_pow2(std::max(1, std::min(16, kColLdsElems / ny)))); }
int multi_cols_max(int ny, int tw) {
  return std::min(tw, floor_pow2(std::max(1, std::min(16, kColLdsElems / (kMultiSlots * ny)))));
}

ColPlan default_plan(int ny, int tw) { return ColPlan{conv_cols_max(ny, tw), multi_cols_max(ny, tw), 16, 16}; }

bool plan_ok(const ColPlan& p, int ny, int tw) {
  auto cw_ok = [&](int cw, int mx) { return cw >= 1 && is_pow2(cw) && cw <= mx; };
  auto radix_ok = [](int r) { return r == 8 || r == 16; };
  return cw_ok(p.conv_cw, conv_cols_max(ny, tw)) && cw_ok(p.multi_cw, multi_cols_max(ny, tw)) &&
         radix_ok(p.conv_radix) && radix_ok(p.multi_radix);
}

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
  if (c->filter_order < 0 || c->filter_order > 6) return false;
  // the nine-point Laplacian of the NPS stencils is defined on a square lattice
  if (c->filter_order == 6 && c->dx != c->dy) return false;
  if (c->precision != 0 && c->precision != 1) return false;
  if (c->convection < 0 || c->convection > 4) return false;
  // the characteristic lines of the flux limiter have steps dr and sqrt(2) dr
  if (c->convection == 4 && c->dx != c->dy) return false;
  return true;
}

struct Layout {
  size_t f, flo, sf, flr, spec, macro, cpl, twx, twy, kx, ky, scx, scy, pd, pf, gl, total;
};

// Planes of the spectral block (contiguous, so that a column pass addresses them by index).
enum : int { SB_SM = 0, SB_S1 = 4, SB_S2I = 10, SB_S2O = 15, SB_PLANES = 18 };
// With the NPS stencils every stage-1 derivative comes from the column pass: 5 more planes
// after the block (dyux, thx, thy, Tx, Ty follow s1 = rx, ry, lap, dxux, dyux, dxuy).
constexpr int SB_NPS = SB_PLANES, SB_NPS_EXTRA = 5;

size_t align_up(size_t v) { return (v + FFTLB_WORKSPACE_ALIGN - 1) / FFTLB_WORKSPACE_ALIGN * FFTLB_WORKSPACE_ALIGN; }

// Workspace layout of a configuration (a compensated state adds the 33 low-part planes).
Layout make_layout(const fftlb_config& c) {
  const int nx = c.nx, ny = c.ny;
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
  L.flo = take(c.precision == 1 ? 33 * plane : 0);
  L.sf = take(32 * plane);
  L.flr = take(c.convection == 4 ? 32 * plane : 0);
  L.spec = take((SB_PLANES + (c.filter_order == 6 ? SB_NPS_EXTRA : 0)) * plane);
  L.macro = take(4 * plane);
  L.cpl = take(plane);
  L.twx = take((size_t)nx * sizeof(float2));
  L.twy = take((size_t)ny * sizeof(float2));
  L.kx = take((size_t)(nx / 2) * sizeof(float));
  L.ky = take((size_t)ny * sizeof(float));
  L.scx = take((size_t)(nx / 2) * sizeof(float2));
  L.scy = take((size_t)ny * sizeof(float2));
  L.pd = take(nblk * 6 * sizeof(double));
  L.pf = take(nblk * 2 * sizeof(float));
  L.gl = take(FFTLB_NGLOBALS * sizeof(double));
  L.total = o;
  return L;
}

// Windowed wavenumber k_m (Eqs. (44)-(47)) of signed index n on a grid of N points with
// spacing d; the Nyquist index -N/2 gets 0.  m = 0 is the exact wavenumber; m = 5 the
// symbol sin(k d) / d of the second-order central difference (g[J+1] - g[J-1]) / (2 d) of
// Sec. 3.1: on a periodic grid that stencil is multiplication by i sin(k d) / d.
__host__ __device__ double windowed_k(int n, int N, double d, int m) {
  if (2 * n == -N || 2 * n == N) return 0.0;
  const double k = 2.0 * M_PI * n / (N * d);
  if (m == 0) return k;
  // m = 6 (the NPS stencils) never reads these tables; it gets the central-difference values
  if (m == 5 || m == 6) return sin(2.0 * M_PI * (double)n / N) / d;
  const double c[4] = {1.0, 1.0 / 6.0, 3.0 / 40.0, 5.0 / 112.0};
  const double s = sin(M_PI * (double)n / N);
  double acc = 0.0, sp = s;
  for (int j = 0; j < m; ++j) {
    acc += c[j] * sp;
    sp *= s * s;
  }
  return 2.0 / d * acc;
}

ColGroup group(std::initializer_list<int> in, std::initializer_list<int> out,
               std::initializer_list<std::initializer_list<int>> kinds) {
  ColGroup g{};
  g.nin = (int)in.size();
  g.nout = (int)out.size();
  if (!nps_shape_ok(g.nin, g.nout)) throw std::logic_error("derivative group shape without a column-pass body");
  int i = 0;
  for (int p : in) g.in[i++] = p;
  i = 0;
  for (int p : out) g.out[i++] = p;
  i = 0;
  for (auto& row : kinds) {
    int j = 0;
    for (int k : row) g.kind[i][j++] = k;
    ++i;
  }
  return g;
}

// Stage 1: only the y-derivatives need the column pass; x-derivatives are formed in the
// stage-2 row kernel from the moment spectra.  Moment spectra sm = [rho, ux, uy, T];
// s1 = [D_y rho, D_yy rho, D_y ux, D_y uy, D_y theta, D_y T] with D_y theta = D_y D_x ux + D_yy uy.
ColLaunch stage1_groups() {
  ColLaunch a{};
  const int sm = SB_SM, s1 = SB_S1;
  a.g[0] = group({sm}, {s1, s1 + 1}, {{MK_IKY}, {MK_KYY}});
  a.g[1] = group({sm + 1, sm + 2}, {s1 + 2, s1 + 3, s1 + 4}, {{MK_IKY, MK_NONE}, {MK_NONE, MK_IKY}, {MK_KXY, MK_KYY}});
  a.g[2] = group({sm + 3}, {s1 + 5}, {{MK_IKY}});
  return a;
}

// Stage 1 with the NPS stencils (filter_order 6): every derivative in the column pass, since the
// nine-point stencils couple the axes.  s1 = [rx, ry, lap, dxux, dyux, dxuy] and, after the
// block, [dyuy, thx, thy, Tx, Ty]; lap is the nine-point Laplacian, thx and thy are
// compositions of the first derivatives (D_x theta = D_x D_x ux + D_x D_y uy).
ColLaunch stage1_nps_groups() {
  ColLaunch a{};
  const int sm = SB_SM, s1 = SB_S1, sn = SB_NPS;
  a.g[0] = group({sm}, {s1, s1 + 1, s1 + 2}, {{MK_IKX}, {MK_IKY}, {MK_LAP}});
  a.g[1] = group({sm + 1, sm + 2}, {s1 + 3, s1 + 4, s1 + 5}, {{MK_IKX, MK_NONE}, {MK_IKY, MK_NONE}, {MK_NONE, MK_IKX}});
  a.g[2] = group({sm + 1, sm + 2}, {sn, sn + 1, sn + 2}, {{MK_NONE, MK_IKY}, {MK_KXX, MK_KXY}, {MK_KXY, MK_KYY}});
  a.g[3] = group({sm + 3}, {sn + 3, sn + 4}, {{MK_IKX}, {MK_IKY}});
  return a;
}

// Stage 2: B^x = D_x(S + Lxx) + D_y Lxy,  B^y = D_x Lxy + D_y(S + Lyy),  G = D_x gx + D_y gy.
ColLaunch stage2_groups() {
  ColLaunch b{};
  const int i2 = SB_S2I, o2 = SB_S2O;
  b.g[0] = group({i2, i2 + 1, i2 + 2}, {o2, o2 + 1}, {{MK_IKX, MK_IKY, MK_NONE}, {MK_NONE, MK_IKX, MK_IKY}});
  b.g[1] = group({i2 + 3, i2 + 4}, {o2 + 2}, {{MK_IKX, MK_IKY}});
  return b;
}

// fftlb_derivative: spectral plane p -> plane p + 1 through the full 2D pass.
ColLaunch derivative_group(int op, int p) {
  const int kinds[3] = {MK_IKX, MK_IKY, MK_LAP};
  ColLaunch d{};
  d.g[0] = group({p}, {p + 1}, {{kinds[op]}});
  return d;
}

// Residual pass: D.j = D_x j_x + D_y j_y from the momentum spectra in s1 planes 0, 1 into plane 2.
ColLaunch divergence_group() {
  ColLaunch d{};
  d.g[0] = group({SB_S1, SB_S1 + 1}, {SB_S1 + 2}, {{MK_IKX, MK_IKY}});
  return d;
}

const ColLaunch kStage1 = stage1_groups();
const ColLaunch kStage1Nps = stage1_nps_groups();
const ColLaunch kStage2 = stage2_groups();
const ColLaunch kDivJ = divergence_group();

}  // namespace

struct fftlb_handle {
  fftlb_config cfg;
  int device;
  int nx, ny, tw;
  Layout L;
  Inst I;
  const Inst* self;  // &I, as a one-entry instance list
  ColPlan plan;
  int64_t steps;
  hipStream_t cap;         // capture stream
  hipGraphExec_t g[kGraphLevels];  // step graphs of 2^i steps
  // Recorded on the caller's stream after every replay of a step graph: a captured graph is
  // destroyed only after its last replay has finished (set_plan, destroy).
  hipEvent_t replayed;
  bool pending;            // `replayed` was recorded since the last wait on it
  bool graphs_at_init;     // capture the step graphs in fftlb_init and after a plan change
  double* gdev;            // FFTLB_NGLOBALS doubles in the workspace for fftlb_poll
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
// Dispatch over compile-time sizes
// ---------------------------------------------------------------------------

#define FFTLB_FOR_ROW_SIZES(X) \
  X(8) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(2048)
#define FFTLB_FOR_COL_SIZES(X) X(4) FFTLB_FOR_ROW_SIZES(X)

int rows(const StepLaunch& L, int kernel, const Inputs& in, hipStream_t s) {
  switch (L.nx) {
#define X(n) \
  case n: return launch_rows<n>(L, kernel, in, s);
    FFTLB_FOR_ROW_SIZES(X)
#undef X
  }
  return FFTLB_EINVAL;
}

int col_multi(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s) {
  if (L.nps) {
    switch (L.ny) {
#define X(n) \
  case n: return launch_col_nps<n>(L, groups, ngroups, s);
      FFTLB_FOR_COL_SIZES(X)
#undef X
    }
    return FFTLB_EINVAL;
  }
  switch (L.ny) {
#define X(n) \
  case n: return launch_col_multi<n>(L, groups, ngroups, s);
    FFTLB_FOR_COL_SIZES(X)
#undef X
  }
  return FFTLB_EINVAL;
}

int col_conv_multi(const StepLaunch& L, const ColLaunch& groups, int ngroups, int pfirst, int nplanes, hipStream_t s) {
  switch (L.ny) {
#define X(n) \
  case n: return launch_col_conv_multi<n>(L, groups, ngroups, pfirst, nplanes, s);
    FFTLB_FOR_COL_SIZES(X)
#undef X
  }
  return FFTLB_EINVAL;
}

int col_conv_scheme(const StepLaunch& L, hipStream_t s) {
  switch (L.ny) {
#define X(n) \
  case n: return launch_col_conv_scheme<n>(L, s);
    FFTLB_FOR_COL_SIZES(X)
#undef X
  }
  return FFTLB_EINVAL;
}

// Real plane -> packed row spectra, and back, for an instance's grid, twiddles and k_x table.
int rows_forward_real(const Inst& I, int nx, const float* a, float2* sa, hipStream_t s) {
  switch (nx) {
#define X(n) \
  case n: return launch_rows_forward_real<n>(I.nblk, a, nullptr, sa, nullptr, I.P.sg, I.P.twx, s);
    FFTLB_FOR_ROW_SIZES(X)
#undef X
  }
  return FFTLB_EINVAL;
}

int rows_inverse_real(const Inst& I, int nx, const float2* sa, float* a, hipStream_t s) {
  switch (nx) {
#define X(n) \
  case n: return launch_rows_inverse_real<n>(I.nblk, sa, nullptr, a, nullptr, I.P.sg, I.P.twx, I.P.kapx, s);
    FFTLB_FOR_ROW_SIZES(X)
#undef X
  }
  return FFTLB_EINVAL;
}

StepLaunch single_launch(const fftlb_handle* h, const ColPlan& plan) {
  return StepLaunch{&h->self, nullptr, 1,    nullptr,
                    h->nx,    h->ny,   h->tw, h->I.nblk,
                    plan,     h->cfg.precision == 1, h->I.scheme, h->cfg.filter_order == 6};
}

// ---------------------------------------------------------------------------
// The step
// ---------------------------------------------------------------------------

constexpr int kNumStages = 4;
// Kernels of the step, in order, and the stage-1 derivative column pass by itself (the
// diagnostics reuse it; in the step it runs inside a convection launch).
enum : int { ST_CONV_S1 = 0, ST_S2_ROWS = 1, ST_S2_COLS = 2, ST_COLLIDE = 3, ST_S1_COLS = 4 };

// The convection columns of the 24 populations with v_y != 0 are split over the two
// derivative column passes of the step, which are latency-bound and leave most of the GPU
// idle: the first kConvSplit of them run in the stage-1 launch, the rest in the stage-2
// launch.  Measured at 1024^2 (step time against the split 8, 12, 16, 18, 20, 24): 16 is
// best, and 16..20 are within 1 us of each other.
constexpr int kConvSplit = 16;

// The stage-1 derivative column pass by itself: the windowed groups, or with the NPS
// stencils all 11 derivatives.
int stage1_columns(const StepLaunch& L, hipStream_t s) {
  return L.nps ? col_multi(L, kStage1Nps, 4, s) : col_multi(L, kStage1, 3, s);
}

// The flux-limiter convection of every instance of a launch, kSchemeSlots instances per pair of
// launches: the real-space stencil kernel, then the row transforms of its 32 planes into the
// population spectra (which the collide takes as they are).  Two launches per step and group,
// whatever the number of instances, so that batch graphs stay as small as with the other schemes.
int conv_flux_limiter(const StepLaunch& L, hipStream_t s) {
  for (int first = 0; first < L.ninst; first += kSchemeSlots) {
    const int count = std::min(kSchemeSlots, L.ninst - first);
    FlBatch fb{};
    PlaneFwdArgs pf{};
    fb.state = pf.state = L.state;
    for (int k = 0; k < count; ++k) {
      const Inst& I = *L.inst[first + k];
      const int id = L.id ? L.id[first + k] : 0;
      fb.c[k] = I.fl;
      fb.c[k].id = id;
      pf.c[k] = PlaneFwdInst{I.fl.out, I.P.sf, I.P.twx, I.P.sg, (long)L.nx * L.ny, id};
    }
    hipLaunchKernelGGL(k_conv_fl, dim3((L.nx + 255) / 256, L.ny, 32 * count), dim3(256), 0, s, fb);
    switch (L.nx) {
#define X(n) \
  case n: RC_TRY(launch_rows_forward_planes<n>(pf, count, L.nblk, s)); break;
      FFTLB_FOR_ROW_SIZES(X)
#undef X
      default: return FFTLB_EINVAL;
    }
  }
  return FFTLB_OK;
}

// With a finite-difference convection scheme the derivative column passes run by themselves
// and the scheme's convection pass of all 32 moving populations follows the stage-1 pass.
int enqueue_stage(const StepLaunch& L, int stage, hipStream_t s) {
  if (L.scheme == 4) {
    switch (stage) {
      case ST_CONV_S1: RC_TRY(stage1_columns(L, s)); return conv_flux_limiter(L, s);
      case ST_S2_COLS: return col_multi(L, kStage2, 2, s);
    }
  } else if (L.scheme) {
    switch (stage) {
      case ST_CONV_S1: RC_TRY(stage1_columns(L, s)); return col_conv_scheme(L, s);
      case ST_S2_COLS: return col_multi(L, kStage2, 2, s);
    }
  }
  switch (stage) {
    case ST_CONV_S1: return col_conv_multi(L, kStage1, 3, 0, kConvSplit, s);
    case ST_S2_ROWS: return rows(L, RK_STAGE2, Inputs{}, s);
    case ST_S2_COLS: return col_conv_multi(L, kStage2, 2, kConvSplit, 24 - kConvSplit, s);
    case ST_COLLIDE: return rows(L, RK_COLLIDE, Inputs{}, s);
    case ST_S1_COLS: return stage1_columns(L, s);
  }
  return FFTLB_EINVAL;
}

// Residual of the current state: dt max |D.(rho u)| and a non-finite flag, into the
// per-block partials (uses the stage-1 spectral planes, free between steps).
int enqueue_residual(const StepLaunch& L, hipStream_t s) {
  RC_TRY(rows(L, RK_MOMENTUM, Inputs{}, s));
  RC_TRY(col_multi(L, kDivJ, 1, s));
  return rows(L, RK_RESIDUAL, Inputs{}, s);
}

// One step of every launch group in `Ls`, kernel after kernel.  (The convection column
// pass is independent of the derivative column passes; it overlaps them inside joint
// launches, not on concurrent graph branches.)
int enqueue_step_all(const StepLaunch* Ls, int nl, hipStream_t s) {
  for (int k = 0; k < kNumStages; ++k)
    for (int i = 0; i < nl; ++i) RC_TRY(enqueue_stage(Ls[i], k, s));
  return FFTLB_OK;
}

// The capture stream (default priority), created on first use.
int make_stream(hipStream_t* a) {
  if (!*a) HIP_TRY(hipStreamCreateWithFlags(a, hipStreamNonBlocking));
  return FFTLB_OK;
}

// Capture what `body` enqueues on the capture stream into an executable graph.
template <typename Body>
int capture_graph(hipStream_t cap, Body body, hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
  const int rc = body();
  hipError_t le = hipGetLastError();
  hipError_t ee = hipStreamEndCapture(cap, &graph);
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

int capture(fftlb_handle* h, int nsteps, hipGraphExec_t* out) {
  RC_TRY(make_stream(&h->cap));
  const StepLaunch L = single_launch(h, h->plan);
  return capture_graph(
      h->cap,
      [&]() {
        for (int i = 0; i < nsteps; ++i) RC_TRY(enqueue_step_all(&L, 1, h->cap));
        return FFTLB_OK;
      },
      out);
}

// Wait until the last replay of the handle's step graphs has finished.  Destroying an
// executable graph whose launches are still queued or running is not allowed (the runtime
// still reads its nodes and kernel arguments); the plan change of a running solver did
// exactly that before this wait existed.
int wait_replays(fftlb_handle* h) {
  if (h->pending) {
    HIP_TRY(hipEventSynchronize(h->replayed));
    h->pending = false;
  }
  return FFTLB_OK;
}

int drop_graphs(fftlb_handle* h) {
  RC_TRY(wait_replays(h));
  for (hipGraphExec_t& g : h->g)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  return FFTLB_OK;
}

// Capture every step graph that is missing.
int ensure_graphs(fftlb_handle* h) {
  for (int i = 0; i < kGraphLevels; ++i)
    if (!h->g[i]) RC_TRY(capture(h, 1 << i, &h->g[i]));
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

// Recompute every spectrum and the moments from the handle's own f (set-state in place;
// each thread reads and writes only its own sites): restores a consistent state after
// kernels were run out of order.
int refresh_from_f(fftlb_handle* h, hipStream_t s) {
  Inputs in{};
  in.a[0] = h->I.P.f;
  RC_TRY(rows(single_launch(h, h->plan), RK_SET, in, s));
  return check_launch("refresh");
}

// The FP64 globals of the current state into `out` (device, FFTLB_NGLOBALS doubles): the
// stage-1 column pass and the stage-2 row kernel (mass, momentum, energy, max |u|,
// non-finite flag), the residual pass, and the fixed-order final sum.
int enqueue_globals(fftlb_handle* h, double* out, hipStream_t s) {
  const StepLaunch L = single_launch(h, h->plan);
  RC_TRY(enqueue_stage(L, ST_S1_COLS, s));
  RC_TRY(enqueue_stage(L, ST_S2_ROWS, s));
  RC_TRY(enqueue_residual(L, s));
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, h->I.P.part_d, h->I.nblk, h->I.P.part_f, h->I.nblk,
                     h->cfg.dx * h->cfg.dy, h->cfg.dt, (double)h->steps, out);
  return check_launch("globals");
}

// ---------------------------------------------------------------------------
// Plan cache: a text file with one line "arch nx ny conv_cols multi_cols conv_radix
// multi_radix" per grid size and device architecture.
// ---------------------------------------------------------------------------

std::string device_arch(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

bool cache_lookup(const char* path, const std::string& arch, int nx, int ny, ColPlan* out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char a[64];
  int x, y, c, m, rc, rm;
  bool found = false;
  while (std::fscanf(f, "%63s %d %d %d %d %d %d", a, &x, &y, &c, &m, &rc, &rm) == 7)
    if (arch == a && x == nx && y == ny) {
      *out = ColPlan{c, m, rc, rm};
      found = true;  // the last entry for a size wins
    }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& arch, int nx, int ny, const ColPlan& p) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d\n", arch.c_str(), nx, ny, p.conv_cw, p.multi_cw, p.conv_radix,
               p.multi_radix);
  std::fclose(f);
}

// Time of the given stages: after one untimed round, the smallest of three means of
// `reps` rounds (the minimum is robust against other work or clock changes in one trial).
int time_stages(const StepLaunch& L, const int* stages, int ns, int reps, hipStream_t s, hipEvent_t e0,
                hipEvent_t e1, float* ms) {
  for (int k = 0; k < ns; ++k) RC_TRY(enqueue_stage(L, stages[k], s));
  *ms = 1e30f;
  for (int trial = 0; trial < 3; ++trial) {
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r)
      for (int k = 0; k < ns; ++k) RC_TRY(enqueue_stage(L, stages[k], s));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float t;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = std::min(*ms, t / reps);
  }
  return FFTLB_OK;
}

// Time every column plan of the handle's size on its own state and keep the fastest: the
// two joint convection and derivative launches of the step (tile width x radix; their
// derivative tiles follow from them) and the stand-alone derivative passes of the
// diagnostics (tile width x radix, timed on the stage-1 pass) are independent choices.
int tune(fftlb_handle* h, int reps, hipStream_t s, ColPlan* best) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("hipEventCreate", hipErrorUnknown);
    return FFTLB_EHIP;
  }
  const int conv_stages[2] = {ST_CONV_S1, ST_S2_COLS}, multi_stages[1] = {ST_S1_COLS};
  float bc = 1e30f, bm = 1e30f;
  ColPlan b = h->plan;
  int rc = FFTLB_OK;
  for (int radix : {16, 8}) {
    for (int cw = 1; cw <= conv_cols_max(h->ny, h->tw) && rc == FFTLB_OK; cw *= 2) {
      float ms;
      const ColPlan p{cw, h->plan.multi_cw, radix, h->plan.multi_radix};
      rc = time_stages(single_launch(h, p), conv_stages, 2, reps, s, e0, e1, &ms);
      if (rc == FFTLB_OK && ms < bc) bc = ms, b.conv_cw = cw, b.conv_radix = radix;
    }
    for (int cw = 1; cw <= multi_cols_max(h->ny, h->tw) && rc == FFTLB_OK; cw *= 2) {
      float ms;
      const ColPlan p{h->plan.conv_cw, cw, h->plan.conv_radix, radix};
      rc = time_stages(single_launch(h, p), multi_stages, 1, reps, s, e0, e1, &ms);
      if (rc == FFTLB_OK && ms < bm) bm = ms, b.multi_cw = cw, b.multi_radix = radix;
    }
  }
  if (rc == FFTLB_OK) *best = b;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != FFTLB_OK) return rc;
  // the timed launches repeated stages out of order: rebuild the spectra from f
  return refresh_from_f(h, s);
}

// A new plan: the step graphs of the old one are destroyed once their last replay has
// finished, and captured again (now, for a solver that captures at init; else at the next
// step call).
int set_plan(fftlb_handle* h, const ColPlan& p) {
  if (!plan_ok(p, h->ny, h->tw)) return FFTLB_EINVAL;
  if (p.conv_cw != h->plan.conv_cw || p.multi_cw != h->plan.multi_cw || p.conv_radix != h->plan.conv_radix ||
      p.multi_radix != h->plan.multi_radix) {
    RC_TRY(drop_graphs(h));
    h->plan = p;
    if (h->graphs_at_init) RC_TRY(ensure_graphs(h));
  }
  return FFTLB_OK;
}

int autotune(fftlb_handle* h, int reps, const char* cache_path, hipStream_t s, ColPlan* best) {
  const std::string arch = device_arch(h->device);
  ColPlan p;
  if (cache_path && cache_lookup(cache_path, arch, h->nx, h->ny, &p) && plan_ok(p, h->ny, h->tw)) {
    *best = p;
    return set_plan(h, p);
  }
  RC_TRY(tune(h, reps, s, &p));
  if (cache_path) cache_store(cache_path, arch, h->nx, h->ny, p);
  *best = p;
  return set_plan(h, p);
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

struct fftlb_batch {
  int n;
  int device;
  std::vector<fftlb_handle*> inst;
  PollInfo* dpoll;     // n entries: where the poll finds each instance's partials
  BatchState st;
  struct Group {
    int nx, ny, tw, nblk;
    bool comp;
    int scheme;
    bool nps;
    ColPlan plan;
    std::vector<int> members;  // all instances of this size
  };
  std::vector<Group> groups;
  std::vector<int> hstate;     // last read retirement flags
  hipStream_t cap;
  // one capture branch per grid size (up to kBranches): the sizes are independent until
  // the poll, so their kernels may run side by side
  hipStream_t branch[8];
  hipEvent_t fork, join[8];
  hipGraphExec_t graph;
  int graph_poll;              // steps per replay of `graph`
  double graph_tol;
  int graph_consecutive;
};

namespace {

struct BatchLayout {
  size_t poll, state, below, steps, first, resid, total;
  std::vector<size_t> ws;  // per-instance workspace offsets
};

int batch_layout(int n, const fftlb_config* cfgs, BatchLayout* out) {
  BatchLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.poll = take(n * sizeof(PollInfo));
  L.state = take(n * sizeof(int));
  L.below = take(n * sizeof(int));
  L.steps = take(n * sizeof(long long));
  L.first = take(n * sizeof(long long));
  L.resid = take(n * sizeof(double));
  for (int i = 0; i < n; ++i) {
    if (!config_ok(&cfgs[i])) return FFTLB_EINVAL;
    L.ws.push_back(take(make_layout(cfgs[i]).total));
  }
  L.total = o;
  *out = L;
  return FFTLB_OK;
}

// Running instances per grid size: their ids and instance pointers (kept alive in `ids`
// and `ptrs` while the launches are captured) and one launch per size.
void batch_launches(fftlb_batch* b, std::vector<std::vector<int>>* ids, std::vector<std::vector<const Inst*>>* ptrs,
                    std::vector<StepLaunch>* out) {
  ids->assign(b->groups.size(), {});
  ptrs->assign(b->groups.size(), {});
  out->clear();
  for (size_t k = 0; k < b->groups.size(); ++k)
    for (int i : b->groups[k].members)
      if (b->hstate[i] == 0) {
        (*ids)[k].push_back(i);
        (*ptrs)[k].push_back(&b->inst[i]->I);
      }
  for (size_t k = 0; k < b->groups.size(); ++k) {
    const auto& g = b->groups[k];
    if ((*ids)[k].empty()) continue;
    out->push_back(StepLaunch{(*ptrs)[k].data(), (*ids)[k].data(), (int)(*ids)[k].size(), b->st.state, g.nx, g.ny,
                              g.tw, g.nblk, g.plan, g.comp, g.scheme, g.nps});
  }
}

int batch_capture(fftlb_batch* b, int poll, double tol, int consecutive) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  std::vector<std::vector<int>> ids;
  std::vector<std::vector<const Inst*>> ptrs;
  std::vector<StepLaunch> Ls;
  batch_launches(b, &ids, &ptrs, &Ls);
  if (Ls.empty()) return FFTLB_OK;
  RC_TRY(make_stream(&b->cap));
  const int nb = std::min<int>((int)Ls.size(), 8);
  if (!b->fork) HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  for (int k = 0; k < nb; ++k) {
    RC_TRY(make_stream(&b->branch[k]));
    if (!b->join[k]) HIP_TRY(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
  }
  RC_TRY(capture_graph(
      b->cap,
      [&]() {
        // `poll` steps of each grid size on its own branch, then the residual passes and the poll
        HIP_TRY(hipEventRecord(b->fork, b->cap));
        for (int k = 0; k < nb; ++k) HIP_TRY(hipStreamWaitEvent(b->branch[k], b->fork, 0));
        for (size_t c = 0; c < Ls.size(); ++c)
          for (int i = 0; i < poll; ++i) RC_TRY(enqueue_step_all(&Ls[c], 1, b->branch[c % nb]));
        for (int k = 0; k < nb; ++k) {
          HIP_TRY(hipEventRecord(b->join[k], b->branch[k]));
          HIP_TRY(hipStreamWaitEvent(b->cap, b->join[k], 0));
        }
        for (const StepLaunch& L : Ls) RC_TRY(enqueue_residual(L, b->cap));
        hipLaunchKernelGGL(k_batch_poll, dim3(b->n), dim3(256), 0, b->cap, b->dpoll, b->st, poll, tol, consecutive);
        return FFTLB_OK;
      },
      &b->graph));
  b->graph_poll = poll;
  b->graph_tol = tol;
  b->graph_consecutive = consecutive;
  return FFTLB_OK;
}

int read_state(fftlb_batch* b, hipStream_t s, int* running) {
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(b->hstate.data(), b->st.state, b->n * sizeof(int), hipMemcpyDeviceToHost));
  *running = (int)std::count(b->hstate.begin(), b->hstate.end(), 0);
  return FFTLB_OK;
}

// Free what a handle owns (graphs, capture stream, event) and the handle; waits for the
// handle's last graph replay.
void release_handle(fftlb_handle* h) {
  DeviceGuard dg(h->device);
  (void)drop_graphs(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->replayed) (void)hipEventDestroy(h->replayed);
  delete h;
}

// fftlb_init; `graphs`: capture the step graphs now (batch instances, which are advanced by
// the batch's own graph, capture theirs only if they are ever stepped alone).
int init_handle(const fftlb_config* cfg, void* workspace, size_t ws_bytes, const float* rho0, const float* ux0,
                const float* uy0, const float* T0, void* stream, bool graphs, fftlb_handle** out) {
  if (!out) return FFTLB_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg) || !rho0 || !ux0 || !uy0 || !T0) return FFTLB_EINVAL;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % FFTLB_WORKSPACE_ALIGN)) return FFTLB_ENOSPC;
  const Layout L = make_layout(*cfg);
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
  h->plan = default_plan(h->ny, h->tw);
  for (hipGraphExec_t& g : h->g) g = nullptr;
  h->cap = nullptr;
  h->replayed = nullptr;
  h->pending = false;
  h->graphs_at_init = graphs;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return FFTLB_EHIP;
  }
  char* ws = static_cast<char*>(workspace);
  Inst& I = h->I;
  I = Inst{};
  Planes& P = I.P;
  P.f = reinterpret_cast<float*>(ws + L.f);
  P.flo = cfg->precision == 1 ? reinterpret_cast<float*>(ws + L.flo) : nullptr;
  const long hp = (long)h->nx * h->ny / 2;  // complex values per spectral plane
  P.sf = reinterpret_cast<float2*>(ws + L.sf);
  I.spec = reinterpret_cast<float2*>(ws + L.spec);
  P.sm = I.spec + SB_SM * hp;
  P.s1 = I.spec + SB_S1 * hp;
  P.s2i = I.spec + SB_S2I * hp;
  P.s2o = I.spec + SB_S2O * hp;
  P.macro = reinterpret_cast<float*>(ws + L.macro);
  P.cpl = reinterpret_cast<float*>(ws + L.cpl);
  P.twx = reinterpret_cast<const float2*>(ws + L.twx);
  P.kapx = reinterpret_cast<const float*>(ws + L.kx);
  P.part_d = reinterpret_cast<double*>(ws + L.pd);
  P.part_f = reinterpret_cast<float*>(ws + L.pf);
  h->gdev = reinterpret_cast<double*>(ws + L.gl);
  P.nx = h->nx;
  P.ny = h->ny;
  P.plane = (long)h->nx * h->ny;
  P.sg.ny = h->ny;
  P.sg.tw = h->tw;
  P.sg.log2tw = ilog2(h->tw);
  I.twy = reinterpret_cast<const float2*>(ws + L.twy);
  I.kapy = reinterpret_cast<const float*>(ws + L.ky);
  I.nblk = h->ny / row_rows_per_block(h->nx);
  h->self = &h->I;

  Model& M = I.M;
  M.dt = (float)cfg->dt;
  M.omega = std::isinf(cfg->tau) ? 0.0f : (float)(cfg->dt / cfg->tau);
  M.K = (float)cfg->K;
  M.H = (float)cfg->H;
  M.zeta = (float)cfg->zeta;
  M.q = (float)cfg->q;
  M.a = (float)cfg->a;
  M.b = (float)cfg->b;
  M.scale = (float)(1.0 / ((double)h->nx * h->ny));

  // convection by a finite-difference scheme: LW (1), MLW1 = LW + R3 (2), MLW2 = LW + R3 + R4 (3),
  // the flux limiter (4), or with the NPS stencils (filter_order 6 and convection 0) the NPS
  // first derivatives (5)
  I.scheme = cfg->convection ? cfg->convection : cfg->filter_order == 6 ? 5 : 0;
  SchemeInst& S = I.sch;
  S.spec = P.sf;
  S.twy = I.twy;
  S.scx = reinterpret_cast<const float2*>(ws + L.scx);
  S.scy = reinterpret_cast<const float2*>(ws + L.scy);
  S.nx = h->nx;
  S.tw = h->tw;
  S.id = 0;
  S.cfx = (float)(cfg->dt / cfg->dx);
  S.cfy = (float)(cfg->dt / cfg->dy);
  S.r3 = cfg->convection >= 2 ? 1.0f : 0.0f;
  S.r4 = cfg->convection >= 3 ? 1.0f : 0.0f;
  S.sdt = (float)(1.0 / ((double)h->nx * h->ny * cfg->dt));
  S.nps = I.scheme == 5 ? 1 : 0;
  FlArgs& FA = I.fl;
  FA.f = P.f;
  FA.out = cfg->convection == 4 ? reinterpret_cast<float*>(ws + L.flr) : nullptr;
  FA.nx = h->nx;
  FA.ny = h->ny;
  FA.id = 0;
  FA.cf = (float)(cfg->dt / cfg->dx);
  FA.rdr = (float)(1.0 / cfg->dx);
  NpsInst& N = I.nps;
  N.spec = I.spec;
  N.twy = I.twy;
  N.scx = S.scx;
  N.scy = S.scy;
  N.nx = h->nx;
  N.tw = h->tw;
  N.id = 0;
  N.rdx = (float)(1.0 / cfg->dx);
  N.rdy = (float)(1.0 / cfg->dy);
  N.scale = M.scale;

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
  // (sin theta, cos theta - 1) of the finite-difference schemes, theta = 2 pi k / N of the
  // signed index (cos theta - 1 = -2 sin^2(theta / 2) keeps small angles accurate); exactly
  // 0 for the sine at the Nyquist index, so that the multiplier is real there.
  auto sc = [](int k, int N) {
    const int ks = 2 * k < N ? k : k - N;
    const double sh = std::sin(M_PI * ks / N);
    const float sn = 2 * ks == -N ? 0.0f : (float)std::sin(2.0 * M_PI * ks / N);
    return make_float2(sn, (float)(-2.0 * sh * sh));
  };
  std::vector<float2> scx(h->nx / 2), scy(h->ny);
  for (int k = 0; k < h->nx / 2; ++k) scx[k] = sc(k, h->nx);
  for (int k = 0; k < h->ny; ++k) scy[k] = sc(k, h->ny);

  int rc = FFTLB_OK;
  {
    DeviceGuard dg(h->device);
    hipError_t e;
    if ((e = hipMemcpyAsync(ws + L.twx, twx.data(), twx.size() * sizeof(float2), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.twy, twy.data(), twy.size() * sizeof(float2), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.kx, kx.data(), kx.size() * sizeof(float), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.ky, ky.data(), ky.size() * sizeof(float), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.scx, scx.data(), scx.size() * sizeof(float2), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ws + L.scy, scy.data(), scy.size() * sizeof(float2), hipMemcpyHostToDevice, s))) {
      set_error("table upload", e);
      delete h;
      return FFTLB_EHIP;
    }
    Inputs in{};
    in.a[0] = rho0;
    in.a[1] = ux0;
    in.a[2] = uy0;
    in.a[3] = T0;
    rc = rows(single_launch(h, h->plan), RK_INIT, in, s);
    if (rc == FFTLB_OK) rc = check_launch("init kernel");
    if (rc == FFTLB_OK && (e = hipStreamSynchronize(s)) != hipSuccess) {
      set_error("hipStreamSynchronize", e);
      rc = FFTLB_EHIP;
    }
    if (rc == FFTLB_OK && (e = hipEventCreateWithFlags(&h->replayed, hipEventDisableTiming)) != hipSuccess) {
      set_error("hipEventCreateWithFlags", e);
      rc = FFTLB_EHIP;
    }
    // the step graphs are captured here, so that no capture falls inside a caller's timed steps
    if (rc == FFTLB_OK && graphs) rc = ensure_graphs(h);
    if (rc != FFTLB_OK) {
      release_handle(h);
      return rc;
    }
  }
  *out = h;
  return FFTLB_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free windowed derivative (fftlb_derivative_static): the two spectral planes and
// the tables live in a file-scope device array instead of a caller's workspace.
// ---------------------------------------------------------------------------

constexpr long kStaticMaxSites = 1L << 18;  // nx * ny at most (512 x 512)
constexpr size_t kStaticPlane = kStaticMaxSites * sizeof(float);  // a half-spectrum plane
constexpr size_t kStaticTwx = 2 * kStaticPlane;
constexpr size_t kStaticTwy = kStaticTwx + kMaxN * sizeof(float2);
constexpr size_t kStaticKx = kStaticTwy + kMaxN * sizeof(float2);
constexpr size_t kStaticKy = kStaticKx + kMaxN * sizeof(float);
constexpr size_t kStaticBytes = kStaticKy + kMaxN * sizeof(float);
constexpr int kMaxDevices = 64;

// Twiddles exp(-2 pi i j / N) of both axes and the windowed wavenumbers, in FP64, stored FP32
// (the tables fftlb_init computes on the host).
__global__ __launch_bounds__(256) void k_static_tables(float2* twx, float2* twy, float* kx, float* ky, int nx, int ny,
                                                       double dx, double dy, int m) {
  for (int j = blockIdx.x * 256 + threadIdx.x; j < (nx > ny ? nx : ny); j += gridDim.x * 256) {
    double sn, cs;
    if (j < nx) {
      sincospi(2.0 * j / nx, &sn, &cs);
      twx[j] = make_float2((float)cs, (float)-sn);
    }
    if (j < ny) {
      sincospi(2.0 * j / ny, &sn, &cs);
      twy[j] = make_float2((float)cs, (float)-sn);
      ky[j] = (float)windowed_k(j < ny / 2 ? j : j - ny, ny, dy, m);
    }
    if (j < nx / 2) kx[j] = (float)windowed_k(j, nx, dx, m);
  }
}

std::mutex g_static_mu;
unsigned char* g_static_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

// Device address of `scratch` on device `dev` (current), looked up once per device: each GPU
// holds its own copy of the array, and in host code the array's name is only a stand-in.
int static_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return FFTLB_EINVAL;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_static_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_static_ptr[dev];
  return FFTLB_OK;
}

}  // namespace

extern "C" {

int fftlb_workspace_bytes(const fftlb_config* cfg, size_t* bytes) {
  if (!config_ok(cfg) || !bytes) return FFTLB_EINVAL;
  *bytes = make_layout(*cfg).total;
  return FFTLB_OK;
}

int fftlb_init(const fftlb_config* cfg, void* workspace, size_t ws_bytes, const float* rho0, const float* ux0,
               const float* uy0, const float* T0, void* stream, fftlb_handle** out) {
  return init_handle(cfg, workspace, ws_bytes, rho0, ux0, uy0, T0, stream, true, out);
}
int fftlb_step(fftlb_handle* h, int64_t nsteps, void* stream) {
  if (!h || nsteps < 0) return FFTLB_EINVAL;
  if (nsteps == 0) return FFTLB_OK;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  RC_TRY(ensure_graphs(h));
  const hipGraphExec_t top = h->g[kGraphLevels - 1];
  for (int64_t left = nsteps / kStepsPerGraph; left > 0; --left) HIP_TRY(hipGraphLaunch(top, s));
  const int rest = (int)(nsteps % kStepsPerGraph);
  for (int i = kGraphLevels - 2; i >= 0; --i)
    if (rest & (1 << i)) HIP_TRY(hipGraphLaunch(h->g[i], s));
  HIP_TRY(hipEventRecord(h->replayed, s));
  h->pending = true;
  h->steps += nsteps;
  return FFTLB_OK;
}

int fftlb_run_stage(fftlb_handle* h, int32_t stage, int32_t reps, void* stream) {
  if (!h || stage < 0 || stage >= kNumStages || reps < 0) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const StepLaunch L = single_launch(h, h->plan);
  for (int i = 0; i < reps; ++i) RC_TRY(enqueue_stage(L, stage, s));
  if (stage == ST_COLLIDE) h->steps += reps;
  return check_launch("run_stage");
}

int fftlb_moments(fftlb_handle* h, float* rho, float* ux, float* uy, float* T, double* globals, void* stream) {
  if (!h) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t pb = (size_t)h->nx * h->ny * sizeof(float);
  float* outs[4] = {rho, ux, uy, T};
  for (int i = 0; i < 4; ++i)
    if (outs[i])
      HIP_TRY(hipMemcpyAsync(outs[i], h->I.P.macro + (size_t)i * h->nx * h->ny, pb, hipMemcpyDeviceToDevice, s));
  if (globals) RC_TRY(enqueue_globals(h, globals, s));
  return FFTLB_OK;
}

int fftlb_poll(fftlb_handle* h, double* globals, void* stream) {
  if (!h) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double g[FFTLB_NGLOBALS];
  RC_TRY(enqueue_globals(h, h->gdev, s));
  HIP_TRY(hipMemcpyAsync(g, h->gdev, sizeof g, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (globals) std::memcpy(globals, g, sizeof g);
  return g[6] != 0.0 ? FFTLB_EUNSTABLE : FFTLB_OK;
}

int fftlb_match_energy(fftlb_handle* h, double energy, void* stream) {
  if (!h || !std::isfinite(energy)) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long P = (long)h->nx * h->ny;
  float* mac = h->I.P.macro;
  RC_TRY(enqueue_globals(h, h->gdev, s));
  hipLaunchKernelGGL(k_shift_temperature, dim3((int)std::min<long>(1024, (P + 255) / 256)), dim3(256), 0, s,
                     mac + 3 * P, P, h->gdev, energy);
  // f := f^eq of the macroscopic planes (each thread reads its own sites before it writes them)
  Inputs in{};
  for (int c = 0; c < 4; ++c) in.a[c] = mac + c * P;
  RC_TRY(rows(single_launch(h, h->plan), RK_INIT, in, s));
  return check_launch("match_energy");
}

int fftlb_get_state(fftlb_handle* h, float* f, void* stream) {
  if (!h || !f) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  HIP_TRY(hipMemcpyAsync(f, h->I.P.f, (size_t)33 * h->nx * h->ny * sizeof(float), hipMemcpyDeviceToDevice,
                         reinterpret_cast<hipStream_t>(stream)));
  return FFTLB_OK;
}

int fftlb_set_state(fftlb_handle* h, const float* f, void* stream) {
  if (!h || !f) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  Inputs in{};
  in.a[0] = f;
  RC_TRY(rows(single_launch(h, h->plan), RK_SET, in, reinterpret_cast<hipStream_t>(stream)));
  return check_launch("set_state");
}

int fftlb_derivative(fftlb_handle* h, const float* g, float* out, int32_t op, void* stream) {
  if (!h || !g || !out || g == out || op < 0 || op > 2) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float2* src = h->I.P.s1;
  float2* dst = h->I.P.s1 + (long)h->nx * h->ny / 2;
  RC_TRY(rows_forward_real(h->I, h->nx, g, src, s));
  // the derivative entry point runs every operator through the full 2D pass
  RC_TRY(col_multi(single_launch(h, h->plan), derivative_group(op, SB_S1), 1, s));
  RC_TRY(rows_inverse_real(h->I, h->nx, dst, out, s));
  return check_launch("derivative");
}

int fftlb_derivative_static(const fftlb_config* cfg, const float* g, float* out, int32_t op, void* stream) {
  if (!config_ok(cfg) || !g || !out || g == out || op < 0 || op > 2) return FFTLB_EINVAL;
  if (cfg->filter_order == 6) {
    std::snprintf(g_last_error, sizeof g_last_error,
                  "fftlb_derivative_static: the NPS stencils (filter_order 6) are not available here");
    return FFTLB_EINVAL;
  }
  const int nx = cfg->nx, ny = cfg->ny;
  if ((long)nx * ny > kStaticMaxSites) {
    std::snprintf(g_last_error, sizeof g_last_error,
                  "fftlb_derivative_static: nx * ny = %ld exceeds the static scratch maximum of %ld points",
                  (long)nx * ny, kStaticMaxSites);
    return FFTLB_EINVAL;
  }
  int dev;
  HIP_TRY(hipGetDevice(&dev));
  unsigned char* ptr = nullptr;
  RC_TRY(static_scratch(dev, &ptr));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the instance the kernels see: spectral planes 0 and 1, tables, all in the scratch array
  Inst I{};
  I.spec = reinterpret_cast<float2*>(ptr);
  I.P.twx = reinterpret_cast<const float2*>(ptr + kStaticTwx);
  I.twy = reinterpret_cast<const float2*>(ptr + kStaticTwy);
  I.P.kapx = reinterpret_cast<const float*>(ptr + kStaticKx);
  I.kapy = reinterpret_cast<const float*>(ptr + kStaticKy);
  const int tw = tile_width(nx);
  I.P.sg.ny = ny;
  I.P.sg.tw = tw;
  I.P.sg.log2tw = ilog2(tw);
  I.M.scale = (float)(1.0 / ((double)nx * ny));
  I.nblk = ny / row_rows_per_block(nx);
  hipLaunchKernelGGL(k_static_tables, dim3((std::max(nx, ny) + 255) / 256), dim3(256), 0, s,
                     reinterpret_cast<float2*>(ptr + kStaticTwx), reinterpret_cast<float2*>(ptr + kStaticTwy),
                     reinterpret_cast<float*>(ptr + kStaticKx), reinterpret_cast<float*>(ptr + kStaticKy), nx, ny,
                     cfg->dx, cfg->dy, cfg->filter_order);
  const Inst* self = &I;
  const StepLaunch L{&self, nullptr, 1, nullptr, nx, ny, tw, I.nblk, default_plan(ny, tw), false};
  RC_TRY(rows_forward_real(I, nx, g, I.spec, s));
  RC_TRY(col_multi(L, derivative_group(op, 0), 1, s));
  RC_TRY(rows_inverse_real(I, nx, I.spec + (long)nx * ny / 2, out, s));
  return check_launch("derivative_static");
}

int fftlb_get_plan(const fftlb_handle* h, fftlb_plan* plan) {
  if (!h || !plan) return FFTLB_EINVAL;
  *plan = fftlb_plan{h->plan.conv_cw, h->plan.multi_cw, h->plan.conv_radix, h->plan.multi_radix};
  return FFTLB_OK;
}

int fftlb_set_plan(fftlb_handle* h, const fftlb_plan* plan) {
  if (!h || !plan) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  return set_plan(h, ColPlan{plan->conv_cols, plan->multi_cols, plan->conv_radix, plan->multi_radix});
}

int fftlb_autotune(fftlb_handle* h, int32_t reps, const char* cache_path, void* stream, fftlb_plan* best) {
  if (!h || reps < 1 || reps > 10000) return FFTLB_EINVAL;
  DeviceGuard dg(h->device);
  ColPlan p;
  RC_TRY(autotune(h, reps, cache_path, reinterpret_cast<hipStream_t>(stream), &p));
  if (best) *best = fftlb_plan{p.conv_cw, p.multi_cw, p.conv_radix, p.multi_radix};
  return FFTLB_OK;
}

int fftlb_destroy(fftlb_handle* h) {
  if (!h) return FFTLB_EINVAL;
  {
    DeviceGuard dg(h->device);
    // other work of the caller's streams may still read the workspace through the handle's
    // launches; the graphs themselves are waited for by release_handle
    (void)hipDeviceSynchronize();
  }
  release_handle(h);
  return FFTLB_OK;
}

int fftlb_batch_workspace_bytes(int32_t n, const fftlb_config* cfgs, size_t* bytes) {
  if (n < 1 || n > FFTLB_MAX_BATCH || !cfgs || !bytes) return FFTLB_EINVAL;
  BatchLayout L;
  RC_TRY(batch_layout(n, cfgs, &L));
  *bytes = L.total;
  return FFTLB_OK;
}

int fftlb_batch_create(int32_t n, const fftlb_config* cfgs, void* workspace, size_t ws_bytes,
                       const float* const* rho0, const float* const* ux0, const float* const* uy0,
                       const float* const* T0, void* stream, fftlb_batch** out) {
  if (!out) return FFTLB_EINVAL;
  *out = nullptr;
  if (n < 1 || n > FFTLB_MAX_BATCH || !cfgs || !rho0 || !ux0 || !uy0 || !T0) return FFTLB_EINVAL;
  BatchLayout L;
  RC_TRY(batch_layout(n, cfgs, &L));
  for (int i = 0; i < n; ++i)
    if (!rho0[i] || !ux0[i] || !uy0[i] || !T0[i]) return FFTLB_EINVAL;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % FFTLB_WORKSPACE_ALIGN)) return FFTLB_ENOSPC;
  if (ws_bytes < L.total) return FFTLB_ENOSPC;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);

  fftlb_batch* b = new (std::nothrow) fftlb_batch();
  if (!b) return FFTLB_EINVAL;
  b->n = n;
  b->cap = nullptr;
  b->fork = nullptr;
  for (int k = 0; k < 8; ++k) {
    b->branch[k] = nullptr;
    b->join[k] = nullptr;
  }
  b->graph = nullptr;
  b->graph_poll = 0;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return FFTLB_EHIP;
  }
  b->dpoll = reinterpret_cast<PollInfo*>(ws + L.poll);
  b->st.state = reinterpret_cast<int*>(ws + L.state);
  b->st.below = reinterpret_cast<int*>(ws + L.below);
  b->st.steps = reinterpret_cast<long long*>(ws + L.steps);
  b->st.first_below = reinterpret_cast<long long*>(ws + L.first);
  b->st.residual = reinterpret_cast<double*>(ws + L.resid);
  b->hstate.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    const fftlb_config& c = cfgs[i];
    fftlb_handle* h = nullptr;
    const size_t wsz = make_layout(c).total;
    const int rc = init_handle(&c, ws + L.ws[i], wsz, rho0[i], ux0[i], uy0[i], T0[i], stream, false, &h);
    if (rc) {
      fftlb_batch_destroy(b);
      return rc;
    }
    b->inst.push_back(h);
    auto g = std::find_if(b->groups.begin(), b->groups.end(),
                          [&](const fftlb_batch::Group& gg) {
                            return gg.nx == c.nx && gg.ny == c.ny && gg.comp == (c.precision == 1) &&
                                   gg.scheme == h->I.scheme && gg.nps == (c.filter_order == 6);
                          });
    if (g == b->groups.end()) {
      b->groups.push_back(
          fftlb_batch::Group{c.nx, c.ny, h->tw, h->I.nblk, c.precision == 1, h->I.scheme, c.filter_order == 6,
                             h->plan, {}});
      g = b->groups.end() - 1;
    }
    g->members.push_back(i);
  }
  // poll table and bookkeeping: running, no polls below tol, no steps, first_below = -1
  std::vector<PollInfo> hp(n);
  for (int i = 0; i < n; ++i) hp[i] = PollInfo{b->inst[i]->I.P.part_f, b->inst[i]->I.nblk, b->inst[i]->I.M.dt};
  std::vector<int> zi(n, 0);
  std::vector<long long> zl(n, 0), ml(n, -1);
  std::vector<double> zd(n, 0.0);
  DeviceGuard dg(b->device);
  hipError_t e;
  if ((e = hipMemcpyAsync(b->dpoll, hp.data(), n * sizeof(PollInfo), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(b->st.state, zi.data(), n * sizeof(int), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(b->st.below, zi.data(), n * sizeof(int), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(b->st.steps, zl.data(), n * sizeof(long long), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(b->st.first_below, ml.data(), n * sizeof(long long), hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(b->st.residual, zd.data(), n * sizeof(double), hipMemcpyHostToDevice, s)) ||
      (e = hipStreamSynchronize(s))) {
    set_error("batch upload", e);
    fftlb_batch_destroy(b);
    return FFTLB_EHIP;
  }
  *out = b;
  return FFTLB_OK;
}

int fftlb_batch_autotune(fftlb_batch* b, int32_t reps, const char* cache_path, void* stream) {
  if (!b || reps < 1 || reps > 10000) return FFTLB_EINVAL;
  DeviceGuard dg(b->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (auto& g : b->groups) {
    ColPlan p;
    RC_TRY(autotune(b->inst[g.members[0]], reps, cache_path, s, &p));
    g.plan = p;
    for (int i : g.members) RC_TRY(set_plan(b->inst[i], p));
  }
  // the batch graph of the old plans: destroyed once its replays have finished (the
  // autotuner synchronised `s`, where fftlb_batch_run launches it)
  HIP_TRY(hipStreamSynchronize(s));
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  return FFTLB_OK;
}

int fftlb_batch_run(fftlb_batch* b, double tol, int32_t consecutive, int32_t poll_every, int64_t max_steps,
                    void* stream) {
  if (!b || !(tol >= 0.0) || consecutive < 1 || poll_every < 1 || poll_every > kMaxPollEvery || max_steps < 0)
    return FFTLB_EINVAL;
  DeviceGuard dg(b->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int running;
  RC_TRY(read_state(b, s, &running));
  int captured_for = -1;  // running instances the current graph was captured for
  if (b->graph && b->graph_poll == poll_every && b->graph_tol == tol && b->graph_consecutive == consecutive)
    captured_for = running;
  int64_t done = 0;
  while (running > 0 && done < max_steps) {
    if (running != captured_for) {
      RC_TRY(batch_capture(b, poll_every, tol, consecutive));
      captured_for = running;
    }
    // two replays per status read keep the device busy while the host checks
    const int reps = (max_steps - done) > poll_every ? 2 : 1;
    for (int r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(b->graph, s));
    done += (int64_t)reps * poll_every;
    RC_TRY(read_state(b, s, &running));
  }
  // per-instance step counters for the instance handles' globals
  std::vector<long long> steps(b->n);
  HIP_TRY(hipMemcpy(steps.data(), b->st.steps, b->n * sizeof(long long), hipMemcpyDeviceToHost));
  for (int i = 0; i < b->n; ++i) b->inst[i]->steps = steps[i];
  // an instance retired on a non-finite value (read_state left the flags current)
  if (std::count(b->hstate.begin(), b->hstate.end(), 2)) return FFTLB_EUNSTABLE;
  return FFTLB_OK;
}

int fftlb_batch_status(fftlb_batch* b, int64_t* steps, int64_t* steps_to_tol, double* residual, int32_t* state) {
  if (!b) return FFTLB_EINVAL;
  DeviceGuard dg(b->device);
  HIP_TRY(hipDeviceSynchronize());
  std::vector<long long> v(b->n), first(b->n);
  std::vector<int> st(b->n);
  HIP_TRY(hipMemcpy(v.data(), b->st.steps, b->n * sizeof(long long), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(first.data(), b->st.first_below, b->n * sizeof(long long), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(st.data(), b->st.state, b->n * sizeof(int), hipMemcpyDeviceToHost));
  if (residual) HIP_TRY(hipMemcpy(residual, b->st.residual, b->n * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < b->n; ++i) {
    if (steps) steps[i] = v[i];
    if (steps_to_tol) steps_to_tol[i] = st[i] == 1 ? first[i] : -1;
    if (state) state[i] = st[i];
  }
  return FFTLB_OK;
}

int fftlb_batch_instance(fftlb_batch* b, int32_t i, fftlb_handle** h) {
  if (!b || !h || i < 0 || i >= b->n) return FFTLB_EINVAL;
  *h = b->inst[i];
  return FFTLB_OK;
}

int fftlb_batch_destroy(fftlb_batch* b) {
  if (!b) return FFTLB_EINVAL;
  {
    DeviceGuard dg(b->device);
    (void)hipDeviceSynchronize();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (int k = 0; k < 8; ++k) {
      if (b->branch[k]) (void)hipStreamDestroy(b->branch[k]);
      if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
  }
  for (fftlb_handle* h : b->inst) fftlb_destroy(h);
  delete b;
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
