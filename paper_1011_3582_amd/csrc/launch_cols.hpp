// Column-kernel launchers (definitions; see launch.hpp).
#pragma once
#include "launch.hpp"

namespace fftlb {

// Arguments of instances [first, first + count) of a launch: the convection pass works on
// the population spectra, the derivative passes on the spectral block.
inline ColArgs col_args(const StepLaunch& L, int first, int count, bool conv) {
  ColArgs a{};
  a.state = L.state;
  for (int k = 0; k < count; ++k) {
    const Inst& I = *L.inst[first + k];
    a.c[k] = ColInst{conv ? I.P.sf : I.spec, I.twy, I.P.kapx, I.kapy, L.nx, L.tw, L.id ? L.id[first + k] : 0,
                     I.M.scale, reinterpret_cast<const float2*>(I.P.f), (float)(1.0 / I.P.ny)};
  }
  return a;
}

// Columns per derivative tile in the joint launch: the largest power of two not above
// CW / 3 (at least 1), so that from CW = 4 on the three derivative planes fit in the
// convection tile's LDS (the launch allocates the larger of the two).
constexpr int joint_multi_cw(int cw) { return cw >= 12 ? 4 : cw >= 6 ? 2 : 1; }

template <int NY, int CW, int R>
int col_conv_multi_plan(const StepLaunch& L, const ColLaunch& groups, int ngroups, int pfirst, int nplanes,
                        hipStream_t s) {
  constexpr int CWM = joint_multi_cw(CW);
  if constexpr (NY * CW > kColLdsElems || kMultiSlots * NY * CWM > kColLdsElems) {
    return FFTLB_EINVAL;
  } else {
    constexpr int NT = col_threads(NY, CW, R);
    const int nblocks = ngroups * ((L.nx / 2) / CWM) + nplanes * ((L.nx / 2) / CW);
    const size_t lds = (cmax(lds_alloc(NY * CW), lds_alloc(kMultiSlots * NY * CWM)) + NY) * sizeof(float2);
    for (int first = 0; first < L.ninst; first += kColSlots) {
      const int count = cmin(kColSlots, L.ninst - first);
      ConvMultiArgs a{col_args(L, first, count, true), {}};
      for (int k = 0; k < count; ++k) a.mspec[k] = L.inst[first + k]->spec;
      hipLaunchKernelGGL((k_col_conv_multi<NY, CW, NT, R, CWM>), dim3(nblocks, count), dim3(NT), lds, s, a, groups,
                         ngroups, pfirst);
    }
    return FFTLB_OK;
  }
}

template <int NY, int CW, int R>
int col_multi_plan(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s) {
  if constexpr (kMultiSlots * NY * CW > kColLdsElems) {
    return FFTLB_EINVAL;
  } else {
    constexpr int NT = col_threads(NY, CW, R);
    for (int first = 0; first < L.ninst; first += kColSlots) {
      const int count = cmin(kColSlots, L.ninst - first);
      // kMultiSlots planes of CW columns, then the twiddle tables
      hipLaunchKernelGGL((k_col_multi<NY, CW, NT, R>), dim3((L.nx / 2) / CW, ngroups, count), dim3(NT),
                         (lds_alloc(kMultiSlots * NY * CW) + NY) * sizeof(float2), s, col_args(L, first, count, false),
                         groups);
    }
    return FFTLB_OK;
  }
}

template <int NY, int R>
int col_conv_multi_cw(const StepLaunch& L, const ColLaunch& groups, int ngroups, int pfirst, int nplanes,
                      hipStream_t s) {
  switch (L.plan.conv_cw) {
    case 1: return col_conv_multi_plan<NY, 1, R>(L, groups, ngroups, pfirst, nplanes, s);
    case 2: return col_conv_multi_plan<NY, 2, R>(L, groups, ngroups, pfirst, nplanes, s);
    case 4: return col_conv_multi_plan<NY, 4, R>(L, groups, ngroups, pfirst, nplanes, s);
    case 8: return col_conv_multi_plan<NY, 8, R>(L, groups, ngroups, pfirst, nplanes, s);
    case 16: return col_conv_multi_plan<NY, 16, R>(L, groups, ngroups, pfirst, nplanes, s);
  }
  return FFTLB_EINVAL;
}

template <int NY, int R>
int col_multi_cw(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s) {
  switch (L.plan.multi_cw) {
    case 1: return col_multi_plan<NY, 1, R>(L, groups, ngroups, s);
    case 2: return col_multi_plan<NY, 2, R>(L, groups, ngroups, s);
    case 4: return col_multi_plan<NY, 4, R>(L, groups, ngroups, s);
    case 8: return col_multi_plan<NY, 8, R>(L, groups, ngroups, s);
    case 16: return col_multi_plan<NY, 16, R>(L, groups, ngroups, s);
  }
  return FFTLB_EINVAL;
}

template <int NY>
int launch_col_conv_multi(const StepLaunch& L, const ColLaunch& groups, int ngroups, int pfirst, int nplanes,
                          hipStream_t s) {
  switch (L.plan.conv_radix) {
    case 8: return col_conv_multi_cw<NY, 8>(L, groups, ngroups, pfirst, nplanes, s);
    case 16: return col_conv_multi_cw<NY, 16>(L, groups, ngroups, pfirst, nplanes, s);
  }
  return FFTLB_EINVAL;
}

template <int NY>
int launch_col_multi(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s) {
  switch (L.plan.multi_radix) {
    case 8: return col_multi_cw<NY, 8>(L, groups, ngroups, s);
    case 16: return col_multi_cw<NY, 16>(L, groups, ngroups, s);
  }
  return FFTLB_EINVAL;
}

// One plan for every grid size: 4 columns per block (every supported nx/2 is a multiple
// of 4 and of the spectral tile width's divisor 4, and 4 columns of 2048 fit the LDS
// budget) and radix 16.
template <int NY>
int launch_col_conv_scheme(const StepLaunch& L, hipStream_t s) {
  constexpr int CW = 4, R = 16;
  static_assert(NY * CW <= kColLdsElems, "scheme column tile exceeds the LDS budget");
  constexpr int NT = col_threads(NY, CW, R);
  if ((L.nx / 2) % CW || L.tw % CW) return FFTLB_EINVAL;
  const int nblocks = 32 * ((L.nx / 2) / CW);
  const size_t lds = (lds_alloc(NY * CW) + NY) * sizeof(float2);
  for (int first = 0; first < L.ninst; first += kSchemeSlots) {
    const int count = cmin(kSchemeSlots, L.ninst - first);
    SchemeArgs a{};
    a.state = L.state;
    for (int k = 0; k < count; ++k) {
      a.c[k] = L.inst[first + k]->sch;
      a.c[k].id = L.id ? L.id[first + k] : 0;
    }
    hipLaunchKernelGGL((k_col_conv_scheme<NY, CW, NT, R>), dim3(nblocks, count), dim3(NT), lds, s, a);
  }
  return FFTLB_OK;
}

template <int NY>
int launch_col_nps(const StepLaunch& L, const ColLaunch& groups, int ngroups, hipStream_t s) {
  constexpr int R = 16;
  static_assert(kMultiSlots * NY <= kColLdsElems, "NPS column tile exceeds the LDS budget");
  constexpr int NT = col_threads(NY, 1, R);
  for (int g = 0; g < ngroups; ++g)
    if (!nps_shape_ok(groups.g[g].nin, groups.g[g].nout)) return FFTLB_EINVAL;
  const size_t lds = (lds_alloc(kMultiSlots * NY) + NY) * sizeof(float2);
  for (int first = 0; first < L.ninst; first += kSchemeSlots) {
    const int count = cmin(kSchemeSlots, L.ninst - first);
    NpsArgs a{};
    a.state = L.state;
    for (int k = 0; k < count; ++k) {
      a.c[k] = L.inst[first + k]->nps;
      a.c[k].id = L.id ? L.id[first + k] : 0;
    }
    hipLaunchKernelGGL((k_col_nps<NY, NT, R>), dim3(L.nx / 2, ngroups, count), dim3(NT), lds, s, a, groups);
  }
  return FFTLB_OK;
}

#define FFTLB_INSTANTIATE_COLS(NY)                                    \
  template int launch_col_multi<NY>(const StepLaunch&, const ColLaunch&, int, hipStream_t); \
  template int launch_col_conv_multi<NY>(const StepLaunch&, const ColLaunch&, int, int, int, hipStream_t); \
  template int launch_col_conv_scheme<NY>(const StepLaunch&, hipStream_t); \
  template int launch_col_nps<NY>(const StepLaunch&, const ColLaunch&, int, hipStream_t);

}  // namespace fftlb
