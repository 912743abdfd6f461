// Launchers of the solver's kernels.  Each is a template over the grid size, explicitly
// instantiated for every supported size in the kernel translation units (rows_*.hip,
// cols_*.hip, compiled in parallel); the API layer dispatches on the runtime size.
#pragma once
#include <hip/hip_runtime.h>

#include "fftlb.h"
#include "kernels.hpp"

namespace fftlb {

// Column-pass plan of a grid size: spectral columns per block and the largest radix (8 or
// 16) of the column transforms, for the convection pass and for the derivative passes.
struct ColPlan {
  int conv_cw, multi_cw, conv_radix, multi_radix;
};

// Host-side description of one solver instance (pointers into its workspace).
struct Inst {
  Planes P;
  Model M;
  float2* spec;        // spectral block: moment (4), stage-1 (6), stage-2 in (5) and out (3) planes
  const float2* twy;   // column twiddles
  const float* kapy;   // windowed k_y
  int nblk;            // row blocks
  SchemeInst sch;      // convection by a finite-difference scheme (used when scheme != 0)
  int scheme;          // 0: spectral convection; 1, 2, 3: LW, MLW1, MLW2; 4: flux limiter; 5: NPS
  NpsInst nps;         // derivatives by the NPS stencils (used when the launch's nps is set)
  FlArgs fl;           // the flux-limiter convection (scheme 4)
};

// One launch of a step kernel over `ninst` instances of one grid size (split into launches
// of kRowSlots / kColSlots instances).
struct StepLaunch {
  const Inst* const* inst;  // host array of ninst instances
  const int* id;            // host array of ninst instance ids (null: 0)
  int ninst;
  const int* state;         // device array of retired flags (null: none)
  int nx, ny, tw, nblk;
  ColPlan plan;
  bool comp;                // compensated state (every instance of the launch)
  int scheme;               // convection scheme of every instance of the launch (Inst::scheme)
  bool nps;                 // derivatives by the NPS stencils (filter_order 6) in every instance
};

// Block buffers of the column kernels are kept within 64 KB (in float2 elements).
constexpr int kColLdsElems = 8192;

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Threads of a column block: one butterfly of the largest radix per thread and pass.
constexpr int col_threads(int ny, int cw, int radix) { return cmin(1024, cmax(64, ny * cw / radix)); }

template <int NY>
int launch_col_multi(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s);
template <int NY>
int launch_col_conv_multi(const StepLaunch& L, const ColLaunch& groups, int ngroups, int pfirst, int nplanes,
                          hipStream_t s);
// the finite-difference convection pass of all 32 moving populations (StepLaunch::scheme != 0)
template <int NY>
int launch_col_conv_scheme(const StepLaunch& L, hipStream_t s);
// the 32 flux-limiter convection planes of up to kSchemeSlots instances -> their population spectra
template <int NX>
int launch_rows_forward_planes(const PlaneFwdArgs& a, int count, int nblk, hipStream_t s);
// derivative groups with the NPS stencils (StepLaunch::nps)
template <int NY>
int launch_col_nps(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s);

enum : int { RK_STAGE2 = 0, RK_COLLIDE = 1, RK_INIT = 2, RK_SET = 3, RK_MOMENTUM = 4, RK_RESIDUAL = 5 };
template <int NX>
int launch_rows(const StepLaunch& L, int kernel, const Inputs& in, hipStream_t s);
// real plane(s) -> packed row spectra, and back (b / sb may be null)
template <int NX>
int launch_rows_forward_real(int nblk, const float* a, const float* b, float2* sa, float2* sb, SpecGeom sg,
                             const float2* twx, hipStream_t s);
template <int NX>
int launch_rows_inverse_real(int nblk, const float2* sa, const float2* sb, float* a, float* b, SpecGeom sg,
                             const float2* twx, const float* kapx, hipStream_t s);

}  // namespace fftlb
