// Constants and per-site physics of the thermal van der Waals FFT-LB model.
//
//  * velocity set, Eq. (1): v_0 = 0, v_ki = v_k (cos((i-1) pi/4), sin((i-1) pi/4)),
//    v_k = 1.0, 1.9, 2.9, 4.3; population index q = 1 + 8(k-1) + (i-1);
//  * weights F_k(T), Eqs. (4)-(6), evaluated in FP64 per site because the quartic
//    polynomial cancels strongly at liquid-vapour temperatures;
//  * equilibrium, Eq. (3), and force term, Eq. (11), in FP32.
#pragma once
#include <hip/hip_runtime.h>

namespace fftlb {

constexpr int kQ = 33;
constexpr double kSpeeds[4] = {1.0, 1.9, 2.9, 4.3};

struct VelTable {
  float vx[kQ], vy[kQ], v2[kQ];
};

constexpr VelTable make_vel_table() {
  VelTable t{};
  constexpr double r = 0.70710678118654752440;  // cos(pi/4)
  const double c8[8] = {1.0, r, 0.0, -r, -1.0, -r, 0.0, r};
  const double s8[8] = {0.0, r, 1.0, r, 0.0, -r, -1.0, -r};
  t.vx[0] = t.vy[0] = t.v2[0] = 0.0f;
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 8; ++i) {
      const int q = 1 + 8 * k + i;
      t.vx[q] = static_cast<float>(kSpeeds[k] * c8[i]);
      t.vy[q] = static_cast<float>(kSpeeds[k] * s8[i]);
      t.v2[q] = static_cast<float>(kSpeeds[k] * kSpeeds[k]);
    }
  return t;
}

// F_k(T) = T (c0 + T (c1 + T (c2 + T c3))) with, for the cyclic neighbours s1, s2, s3 of
// s_k = v_k^2 (Eq. (6)): c3 = 48/D, c2 = -6 (s1 + s2 + s3)/D, c1 = (s1 s2 + s2 s3 + s3 s1)/D,
// c0 = -s1 s2 s3 / (4 D), D = s_k (s_k - s1)(s_k - s2)(s_k - s3).
struct WeightPoly {
  double c[4][4];
};

constexpr WeightPoly make_weight_poly() {
  WeightPoly w{};
  double s[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k) s[k] = kSpeeds[k] * kSpeeds[k];
  for (int k = 0; k < 4; ++k) {
    const double s1 = s[(k + 1) % 4], s2 = s[(k + 2) % 4], s3 = s[(k + 3) % 4];
    const double D = s[k] * (s[k] - s1) * (s[k] - s2) * (s[k] - s3);
    w.c[k][3] = 48.0 / D;
    w.c[k][2] = -6.0 * (s1 + s2 + s3) / D;
    w.c[k][1] = (s1 * s2 + s2 * s3 + s3 * s1) / D;
    w.c[k][0] = -s1 * s2 * s3 / (4.0 * D);
  }
  return w;
}

// internal linkage: every translation unit that launches kernels holds its own copy
static __constant__ VelTable c_vel = make_vel_table();
static __constant__ WeightPoly c_wpoly = make_weight_poly();

// Scalar parameters handed to the kernels by value.
struct Model {
  float dt;     // time step
  float omega;  // dt / tau (0 when the collision is off)
  float K, H, zeta, q, a, b;
  float scale;  // 1 / (nx ny): normalisation of the inverse 2D transform
};

// Weight F_k(T) of speed group k (0-based), Eq. (4), in FP64.
__device__ __forceinline__ double group_weight(double t, int k) {
  const double* c = c_wpoly.c[k];
  return t * (c[0] + t * (c[1] + t * (c[2] + t * c[3])));
}

// Weight of the rest particle, Eq. (5): F_0 = 1 - 8 (F_1 + F_2 + F_3 + F_4).
__device__ __forceinline__ float rest_weight(float T) {
  const double t = T;
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) sum += group_weight(t, k);
  return static_cast<float>(1.0 - 8.0 * sum);
}

// What the 33-velocity loop keeps per site: the moments and the force polynomial
// A + B.(v-u) + (C+Cq)|v-u|^2 = s0 + sx vx + sy vy + cc |v|^2 (Eqs. (11), (20)), the
// latter with -dt folded in for the update.
struct Site {
  float rho, ux, uy, T;
  float uxT, uyT;   // u / T
  float s0, cc;     // velocity-independent part and |v|^2 coefficient of the force polynomial
  float dsx, dsy;   // -dt sx, -dt sy
};

// Per-site factors of Eq. (3) for one speed group: with w = v.u/T, f^eq = rho F_k (base +
// g w + (g/2) w^2 + w^3/6 + w^4/24), g = 1 - u^2/2T, base = g + u^4/8T^2; the rho F_k
// factor is folded into the five coefficients (Horner form).
struct GroupEq {
  float c0, c1, c2, c3, c4;
};

__device__ __forceinline__ void site_init(Site& s, float rho, float ux, float uy, float T) {
  s.rho = rho;
  s.ux = ux;
  s.uy = uy;
  s.T = T;
  const float iT = 1.0f / T;
  s.uxT = ux * iT;
  s.uyT = uy * iT;
  s.s0 = s.cc = s.dsx = s.dsy = 0.0f;
}

// Force coefficients A, B, C + C_q (Eqs. (20)-(23)) folded into the polynomial in v.
__device__ __forceinline__ void site_force(Site& s, const Model& M, float Bx, float By, float cc) {
  const float A = -2.0f * cc * s.T;
  const float u2 = s.ux * s.ux + s.uy * s.uy;
  s.s0 = A - (Bx * s.ux + By * s.uy) + cc * u2;
  s.dsx = -M.dt * (Bx - 2.0f * cc * s.ux);
  s.dsy = -M.dt * (By - 2.0f * cc * s.uy);
  s.cc = cc;
}

__device__ __forceinline__ GroupEq group_eq(const Site& s, float Fk) {
  const float u2T = s.ux * s.uxT + s.uy * s.uyT;  // u^2 / T
  const float g = 1.0f - 0.5f * u2T;
  const float base = g + 0.125f * u2T * u2T;
  const float rF = s.rho * Fk;
  GroupEq e;
  e.c0 = rF * base;
  e.c1 = rF * g;
  e.c2 = 0.5f * e.c1;
  e.c3 = rF * (1.0f / 6.0f);
  e.c4 = rF * (1.0f / 24.0f);
  return e;
}

// Eq. (3) for a moving population with velocity (vx, vy).
__device__ __forceinline__ float feq_moving(const Site& s, const GroupEq& e, float vx, float vy) {
  const float w = fmaf(vx, s.uxT, vy * s.uyT);
  return fmaf(w, fmaf(w, fmaf(w, fmaf(w, e.c4, e.c3), e.c2), e.c1), e.c0);
}

// Eq. (3) for the rest particle (v = 0).
__device__ __forceinline__ float feq_rest(const Site& s) { return group_eq(s, rest_weight(s.T)).c0; }

// -dt times the velocity-independent part of the force polynomial for speed v^2.
__device__ __forceinline__ float force_k0(const Site& s, const Model& M, float v2) {
  return -M.dt * fmaf(s.cc, v2, s.s0);
}

// f^{n+1} = f - dt C - omega (f - feq) + dt I with I = -(s0 + sx vx + sy vy + cc |v|^2) feq,
// k0 = force_k0(v^2).  The increment is formed first and added once: f is rounded to FP32
// a single time and no O(eps) multiple of f (e.g. from rounding 1 - omega) biases the mass.
__device__ __forceinline__ float relax_increment(const Site& s, const Model& M, float f, float feq, float conv,
                                                 float vx, float vy, float k0) {
  const float kf = fmaf(s.dsx, vx, fmaf(s.dsy, vy, k0));  // -dt (s0 + sx vx + sy vy + cc v^2)
  return fmaf(M.omega, feq - f, fmaf(kf, feq, -M.dt * conv));
}

__device__ __forceinline__ float relax_update(const Site& s, const Model& M, float f, float feq, float conv,
                                              float vx, float vy, float k0) {
  return f + relax_increment(s, M, f, feq, conv, vx, vy, k0);
}

// The same update of a compensated state f = hi + lo (|lo| <= half an ulp of hi): the
// increment (formed from hi) is added to lo first, and the rounding error of adding the
// result to hi is kept as the new lo (Fast2Sum: exact because |hi| exceeds the addend), so
// increments below half an ulp of f accumulate instead of being lost.  Returns (hi, lo).
__device__ __forceinline__ float2 relax_update_comp(const Site& s, const Model& M, float hi, float lo, float feq,
                                                    float conv, float vx, float vy, float k0) {
  const float t = lo + relax_increment(s, M, hi, feq, conv, vx, vy, k0);
  const float h = hi + t;
  return make_float2(h, t - (h - hi));
}

}  // namespace fftlb
