// Row-kernel launchers (definitions; see launch.hpp).
#pragma once
#include "launch.hpp"

namespace fftlb {

inline RowArgs row_args(const StepLaunch& L, int first, int count) {
  RowArgs a{};
  a.state = L.state;
  for (int k = 0; k < count; ++k) {
    const Inst& I = *L.inst[first + k];
    a.P[k] = I.P;
    a.M[k] = I.M;
    a.id[k] = L.id ? L.id[first + k] : 0;
  }
  return a;
}

template <int NX>
int launch_rows(const StepLaunch& L, int kernel, const Inputs& in, hipStream_t s) {
  using G = RowGeom<NX>;
  const size_t lds = G::LDS_TOTAL * sizeof(float2);
  if (kernel < RK_STAGE2 || kernel > RK_RESIDUAL) return FFTLB_EINVAL;
  for (int first = 0; first < L.ninst; first += kRowSlots) {
    const int count = cmin(kRowSlots, L.ninst - first);
    const dim3 grid(L.nblk, count), block(G::NT);
    const RowArgs a = row_args(L, first, count);
    switch (kernel) {
      case RK_STAGE2:
        if (L.nps)
          hipLaunchKernelGGL((k_rows_stage2<NX, true>), grid, block, G::LDS * sizeof(float2), s, a);
        else
          hipLaunchKernelGGL((k_rows_stage2<NX, false>), grid, block, G::LDS * sizeof(float2), s, a);
        break;
      case RK_COLLIDE:
        if (L.scheme && L.comp)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_STEP, true, true>), grid, block, lds, s, a, in);
        else if (L.scheme)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_STEP, false, true>), grid, block, lds, s, a, in);
        else if (L.comp)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_STEP, true>), grid, block, lds, s, a, in);
        else
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_STEP, false>), grid, block, lds, s, a, in);
        break;
      // init and set take the variant of the instance's scheme (the finite-difference schemes
      // need the row spectra of every population; the spectral derivative needs none)
      case RK_INIT:
        if (L.scheme && L.comp)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_INIT, true, true>), grid, block, lds, s, a, in);
        else if (L.scheme)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_INIT, false, true>), grid, block, lds, s, a, in);
        else if (L.comp)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_INIT, true>), grid, block, lds, s, a, in);
        else
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_INIT, false>), grid, block, lds, s, a, in);
        break;
      case RK_SET:
        if (L.scheme && L.comp)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_SET, true, true>), grid, block, lds, s, a, in);
        else if (L.scheme)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_SET, false, true>), grid, block, lds, s, a, in);
        else if (L.comp)
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_SET, true>), grid, block, lds, s, a, in);
        else
          hipLaunchKernelGGL((k_rows_collide<NX, MODE_SET, false>), grid, block, lds, s, a, in);
        break;
      case RK_MOMENTUM: hipLaunchKernelGGL(k_rows_momentum<NX>, grid, block, lds, s, a); break;
      case RK_RESIDUAL: hipLaunchKernelGGL(k_rows_residual<NX>, grid, block, lds, s, a); break;
    }
  }
  return FFTLB_OK;
}

template <int NX>
int launch_rows_forward_real(int nblk, const float* a, const float* b, float2* sa, float2* sb, SpecGeom sg,
                             const float2* twx, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_forward_real<NX>, dim3(nblk), dim3(RowGeom<NX>::NT),
                     RowGeom<NX>::LDS_TOTAL * sizeof(float2), s, a, b, sa, sb, sg, twx, NX);
  return FFTLB_OK;
}

template <int NX>
int launch_rows_inverse_real(int nblk, const float2* sa, const float2* sb, float* a, float* b, SpecGeom sg,
                             const float2* twx, const float* kapx, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_inverse_real<NX>, dim3(nblk), dim3(RowGeom<NX>::NT),
                     RowGeom<NX>::LDS_TOTAL * sizeof(float2), s, sa, sb, a, b, sg, twx, kapx, NX);
  return FFTLB_OK;
}

template <int NX>
int launch_rows_forward_planes(const PlaneFwdArgs& a, int count, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_rows_forward_planes<NX>, dim3(nblk, 16, count), dim3(RowGeom<NX>::NT),
                     RowGeom<NX>::LDS_TOTAL * sizeof(float2), s, a);
  return FFTLB_OK;
}

#define FFTLB_INSTANTIATE_ROWS(NX)                                                                       \
  template int launch_rows<NX>(const StepLaunch&, int, const Inputs&, hipStream_t);                    \
  template int launch_rows_forward_real<NX>(int, const float*, const float*, float2*, float2*, SpecGeom, \
                                            const float2*, hipStream_t);                                 \
  template int launch_rows_inverse_real<NX>(int, const float2*, const float2*, float*, float*, SpecGeom, \
                                            const float2*, const float*, hipStream_t);           \
  template int launch_rows_forward_planes<NX>(const PlaneFwdArgs&, int, int, hipStream_t);

}  // namespace fftlb
