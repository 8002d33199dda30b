// The body-centre split of the pair distance for the FP32 pair kernels (vector-unit and
// matrix-core): constants, the phi evaluation, and the host-side set-up.
#pragma once
#include <cmath>

#include <hip/hip_runtime.h>

#include "phi.h"

namespace mfs {

// ---------------------------------------------------------------------------
// G_hat in FP32 with the distance split at the body centres.
//
// For target i on body a and source j on body b, x_i - x_j = (c_a - c_b) + (l_i - l_j), with
// body-local offsets l (|l| <= body radius) and centre difference dc.  With D = |dc| and
// u = |dl|^2 + 2 dc.dl, the distance is r = D + delta, delta = u / (D + r).  u is evaluated as
// A + |l_j|^2 + P . l_j with A = |l_i|^2 + 2 dc.l_i and P = -2 (l_i + dc) formed once per
// (target, source body) and |l_j|^2 stored per point.  D and the phase
// kappa D mod 2 pi are formed in FP64 once per (target, source body); delta, and with it the
// phase correction, is an O(1) quantity formed in FP32 to ~1e-7 relative.  The phase kappa r is
// therefore accurate to ~1e-6 rad instead of ~kappa r 2^-24 (1e-4 rad at kappa r = 1400).
// Per source body the FP32 partial sums are added into FP64 accumulators, which removes the
// O(sqrt(N) eps) growth of one long FP32 sum.
//
// 2D kernel, three branches on z = kappa r:
//   z >= 12: Hankel modulus and phase expansions (DLMF 10.18.17-18, series of M^2 taken to its
//            square root), 3 terms each: H0 = M e^{i theta},
//            M sqrt(pi z / 2) = 1 - 1/(16 z^2) + 53/(512 z^4),
//            theta = z - pi/4 - 1/(8 z) + 25/(384 z^3) - 1073/(5120 z^5);
//            errors <= 2e-7 (modulus) and 4e-8 rad (phase) for z >= 12;
//   3 <= z < 12: A&S 9.4.3 with the same accurate phase;
//   z < 3: A&S 9.4.1 / 9.4.2.
// 3D kernel: exp(i kappa r) / (4 pi r) with the same phase split.
// ---------------------------------------------------------------------------
struct BodyPhaseConsts {
  float kappa_rev;   // kappa / 2 pi
  float r_far;       // 12 / kappa
  float r_mid;       // 3 / kappa
  // far branch, amplitude (1/4) sqrt(2/(pi kappa)) r^{-1/2} (m0 + m1 r^-2 + m2 r^-4)
  float m0, m1, m2;
  // far branch, phase correction in revolutions: r^-1 (p0 + p1 r^-2 + p2 r^-4)
  float p0, p1, p2;
  // A&S branches
  Phi2DConstsF32 as;
  double kappa_rev64;
  float far_D;       // centre distance beyond which every pair of two bodies has z >= 12
  float vfar_D;      // centre distance beyond which every pair has z >= 100 (shorter expansions)
  float amp3;        // 3D amplitude factor 1 / (4 pi) (times a scale where a kernel wants one)
};


// FAR: 0 = any distance (branches), 1 = every pair has z >= 12, 2 = every pair has z >= 100, where
// the z^-4 modulus term (< 1e-9 relative) and the z^-5 phase term (< 2e-11 rad) are dropped.
template <int DIM, int FAR = 0>
__device__ __forceinline__ void bp_phi(const BodyPhaseConsts& k, float u, float D, float D2, float ph0,
                                       float& pr, float& pi) {
  const float r2 = D2 + u;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  // delta = r - D = u / (D + r), accurate where r >> 1
  const float delta = u * __builtin_amdgcn_rcpf(D + r);
  if constexpr (DIM == 3) {
    const float rev = __builtin_amdgcn_fractf(fmaf(delta, k.kappa_rev, ph0));
    const float a = rinv * k.amp3;  // 1 / (4 pi r)
    pr = a * __builtin_amdgcn_cosf(rev);
    pi = a * __builtin_amdgcn_sinf(rev);
  } else {
    if (FAR > 0 || r >= k.r_far) {
      const float w2 = rinv * rinv;
      const float m = FAR == 2 ? fmaf(k.m1, w2, k.m0) : fmaf(fmaf(k.m2, w2, k.m1), w2, k.m0);
      const float th = FAR == 2 ? rinv * fmaf(k.p1, w2, k.p0) : rinv * fmaf(fmaf(k.p2, w2, k.p1), w2, k.p0);
      const float rev = __builtin_amdgcn_fractf(fmaf(delta, k.kappa_rev, ph0) + th);
      const float a = m * __builtin_amdgcn_sqrtf(rinv);
      // (i/4) H0 = (i/4) M e^{i theta}: re = -A sin, im = A cos
      pr = -a * __builtin_amdgcn_sinf(rev);
      pi = a * __builtin_amdgcn_cosf(rev);
    } else if (r >= k.r_mid) {
      const float t = k.as.three_over_kappa * rinv;
      float f0 = 0.00014476f;
      f0 = fmaf(f0, t, -0.00072805f);
      f0 = fmaf(f0, t, 0.00137237f);
      f0 = fmaf(f0, t, -0.00009512f);
      f0 = fmaf(f0, t, -0.00552740f);
      f0 = fmaf(f0, t, -0.00000077f);
      f0 = fmaf(f0, t, 0.79788456f);
      float th = 0.00013558f * 0.15915494309189535f;
      th = fmaf(th, t, -0.00029333f * 0.15915494309189535f);
      th = fmaf(th, t, -0.00054125f * 0.15915494309189535f);
      th = fmaf(th, t, 0.00262573f * 0.15915494309189535f);
      th = fmaf(th, t, -0.00003954f * 0.15915494309189535f);
      th = fmaf(th, t, -0.04166397f * 0.15915494309189535f);
      th = th * t;  // -1/8 is already in ph0
      const float rev = __builtin_amdgcn_fractf(fmaf(delta, k.kappa_rev, ph0) + th);
      const float a = k.as.amp * f0 * __builtin_amdgcn_sqrtf(rinv);
      pr = -a * __builtin_amdgcn_sinf(rev);
      pi = a * __builtin_amdgcn_cosf(rev);
    } else {
      phi2d_f32(r2, k.as, pr, pi);
    }
  }
}


inline Phi2DConstsF32 make_phi2d_f32(double kappa) {
  Phi2DConstsF32 c;
  c.kappa = (float)kappa;
  c.kappa_rev = (float)(kappa / (2.0 * M_PI));
  c.three_over_kappa = (float)(3.0 / kappa);
  c.amp = (float)(0.25 / std::sqrt(kappa));
  c.kappa2_9 = (float)(kappa * kappa / 9.0);
  c.log_half_kappa = (float)std::log(0.5 * kappa);
  return c;
}

// The far-branch amplitudes (2D expansion coefficients m0..m2, 3D 1/(4 pi)) times 2^shift: phi
// comes out scaled by 2^shift at no cost where every pair takes the far branch.
inline BodyPhaseConsts scale_far_amplitude(BodyPhaseConsts k, int shift) {
  k.m0 = std::ldexp(k.m0, shift);
  k.m1 = std::ldexp(k.m1, shift);
  k.m2 = std::ldexp(k.m2, shift);
  k.amp3 = std::ldexp(k.amp3, shift);
  return k;
}

inline BodyPhaseConsts make_bodyphase(double kappa, double rho_max) {
  BodyPhaseConsts k{};
  const double two_pi = 2.0 * M_PI;
  k.kappa_rev = (float)(kappa / two_pi);
  k.kappa_rev64 = kappa / two_pi;
  k.r_far = (float)(12.0 / kappa);
  k.r_mid = (float)(3.0 / kappa);
  const double amp = 0.25 * std::sqrt(2.0 / (M_PI * kappa));  // (1/4) sqrt(2/(pi kappa))
  const double k2 = kappa * kappa;
  k.m0 = (float)amp;
  k.m1 = (float)(-amp / (16.0 * k2));
  k.m2 = (float)(amp * 53.0 / (512.0 * k2 * k2));
  k.p0 = (float)(-1.0 / (8.0 * kappa) / two_pi);
  k.p1 = (float)(25.0 / (384.0 * k2 * kappa) / two_pi);
  k.p2 = (float)(-1073.0 / (5120.0 * k2 * k2 * kappa) / two_pi);
  k.as = make_phi2d_f32(kappa);
  // |x_i - x_j| >= D - 2 rho_max, so D >= 12/kappa + 2 rho_max (plus rounding slack) is far for all pairs
  k.far_D = (float)((12.0 / kappa + 2.0 * rho_max) * (1.0 + 1e-5) + 1e-6);
  k.vfar_D = (float)((100.0 / kappa + 2.0 * rho_max) * (1.0 + 1e-5) + 1e-6);
  k.amp3 = (float)(1.0 / (4.0 * M_PI));
  return k;
}

}  // namespace mfs
