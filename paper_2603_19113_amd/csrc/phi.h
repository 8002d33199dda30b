// Device evaluation of the Helmholtz fundamental solution (eq. FundamentalSol):
//   2D: phi(x) = (i/4) H_0^(1)(kappa |x|)         3D: phi(x) = exp(i kappa |x|) / (4 pi |x|)
//
// FP32, 2D: Abramowitz & Stegun 9.4.1-9.4.3 polynomial approximations
//   (|eps| <= 5e-8 absolute for z <= 3; f0 and theta0 errors <= 1.6e-8 / 7e-8 for z >= 3),
//   hardware rsq/sqrt, and v_sin/v_cos on a revolution-reduced phase.
// FP64, 2D: power series for J0 and Y0 (DLMF 10.2.2, 10.8.2) for z < 2; Miller's backward
//   recurrence for J_n normalised by the generating-function identity 1 = J0 + 2 sum J_2k, with
//   Neumann's expansion of Y0 in even-order J_n (both in DLMF ch. 10) for 2 <= z < 25; the Hankel
//   asymptotic expansion (DLMF 10.17.5) with 16 terms for z >= 25.  Relative error of H0
//   <= 2e-15 over (0, 2000] in a float64 model checked against mpmath.
// 3D: closed form in either precision.
#pragma once
#include <hip/hip_runtime.h>

namespace mfs {

// ------------------------------------------------------------------ FP32 ---
struct Phi2DConstsF32 {
  float kappa;       // wavenumber
  float kappa_rev;   // kappa / (2 pi): phase in revolutions per unit distance
  float three_over_kappa;
  float amp;         // 1 / (4 sqrt(kappa)): (i/4) H0 far amplitude factor before f0 r^{-1/2}
  float kappa2_9;    // kappa^2 / 9: (z/3)^2 = r^2 kappa^2 / 9
  float log_half_kappa;  // ln(kappa / 2)
};

// phi(r) for 2D, FP32, from r^2. Returns (re, im).
__device__ __forceinline__ void phi2d_f32(float r2, const Phi2DConstsF32& c, float& pr, float& pi) {
  const float rinv = __builtin_amdgcn_rsqf(r2);  // 1 / r
  const float r = r2 * rinv;
  const float z = c.kappa * r;
  if (z >= 3.0f) {
    // A&S 9.4.3: J0 + i Y0 = z^{-1/2} f0 e^{i theta0}, t = 3/z.
    const float t = c.three_over_kappa * rinv;
    float f0 = 0.00014476f;
    f0 = fmaf(f0, t, -0.00072805f);
    f0 = fmaf(f0, t, 0.00137237f);
    f0 = fmaf(f0, t, -0.00009512f);
    f0 = fmaf(f0, t, -0.00552740f);
    f0 = fmaf(f0, t, -0.00000077f);
    f0 = fmaf(f0, t, 0.79788456f);
    // theta0 - z, in revolutions: (-0.78539816 + poly(t)) / (2 pi)
    float th = 0.00013558f * 0.15915494309189535f;
    th = fmaf(th, t, -0.00029333f * 0.15915494309189535f);
    th = fmaf(th, t, -0.00054125f * 0.15915494309189535f);
    th = fmaf(th, t, 0.00262573f * 0.15915494309189535f);
    th = fmaf(th, t, -0.00003954f * 0.15915494309189535f);
    th = fmaf(th, t, -0.04166397f * 0.15915494309189535f);
    th = fmaf(th, t, -0.125f);  // -pi/4 / (2 pi)
    const float rev = __builtin_amdgcn_fractf(fmaf(r, c.kappa_rev, th));
    const float s = __builtin_amdgcn_sinf(rev);
    const float co = __builtin_amdgcn_cosf(rev);
    // (i/4) A e^{i theta}: re = -A/4 sin, im = A/4 cos, A/4 = amp f0 r^{-1/2}
    const float a = c.amp * f0 * __builtin_amdgcn_sqrtf(rinv);
    pr = -a * s;
    pi = a * co;
  } else {
    // A&S 9.4.1 / 9.4.2 in u = (z/3)^2
    const float u = r2 * c.kappa2_9;
    float j0 = 0.0002100f;
    j0 = fmaf(j0, u, -0.0039444f);
    j0 = fmaf(j0, u, 0.0444479f);
    j0 = fmaf(j0, u, -0.3163866f);
    j0 = fmaf(j0, u, 1.2656208f);
    j0 = fmaf(j0, u, -2.2499997f);
    j0 = fmaf(j0, u, 1.0f);
    float y0 = -0.00024846f;
    y0 = fmaf(y0, u, 0.00427916f);
    y0 = fmaf(y0, u, -0.04261214f);
    y0 = fmaf(y0, u, 0.25300117f);
    y0 = fmaf(y0, u, -0.74350384f);
    y0 = fmaf(y0, u, 0.60559366f);
    y0 = fmaf(y0, u, 0.36746691f);
    // ln(z/2) = 0.5 ln(r^2) + ln(kappa/2)
    const float lz = fmaf(0.5f * 0.69314718055994531f, __builtin_amdgcn_logf(r2), c.log_half_kappa);
    y0 = fmaf(0.63661977236758134f * lz, j0, y0);
    pr = -0.25f * y0;
    pi = 0.25f * j0;
  }
}

struct Phi3DConstsF32 {
  float kappa_rev;  // kappa / (2 pi)
};

__device__ __forceinline__ void phi3d_f32(float r2, const Phi3DConstsF32& c, float& pr, float& pi) {
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * rinv;
  const float rev = __builtin_amdgcn_fractf(r * c.kappa_rev);
  const float a = rinv * 0.07957747154594767f;  // 1 / (4 pi r)
  pr = a * __builtin_amdgcn_cosf(rev);
  pi = a * __builtin_amdgcn_sinf(rev);
}

// ------------------------------------------------------------------ FP64 ---
struct PhiConstsF64 {
  double kappa;
};

// Hankel expansion coefficients a_k(0) = (-1)^k prod_{i<=k} (2i-1)^2 / (k! 8^k) (DLMF 10.17.1),
// built at compile time from a_k / a_{k-1} = -(2k-1)^2 / (8k).  With i^k a_k(0) sorted into real
// and imaginary parts: H0 = sqrt(2/(pi z)) e^{i(z - pi/4)} (P + i Q), where
// P = sum_j (-1)^j |a_2j| z^{-2j} and Q = -sum_j (-1)^j |a_{2j+1}| z^{-2j-1}.
struct HankelAsymTable {
  double p[8];  // coefficients of w^{2j} in P, w = 1/z
  double q[8];  // coefficients of w^{2j+1} in Q
};

constexpr HankelAsymTable make_hankel_asym_table() {
  HankelAsymTable t{};
  double a = 1.0;  // |a_k|
  for (int k = 0; k < 16; ++k) {
    if (k > 0) a = a * (double)((2 * k - 1) * (2 * k - 1)) / (8.0 * k);
    const int j = k / 2;
    const double sgn = (j % 2 == 0) ? 1.0 : -1.0;
    if (k % 2 == 0) t.p[j] = sgn * a;
    else t.q[j] = -sgn * a;
  }
  return t;
}

static constexpr HankelAsymTable kHankelAsym = make_hankel_asym_table();

__device__ __forceinline__ void hankel0_asym(double z, double& J, double& Y) {
  const double w = 1.0 / z;
  const double w2 = w * w;
  double P = kHankelAsym.p[7];
#pragma unroll
  for (int i = 6; i >= 0; --i) P = fma(P, w2, kHankelAsym.p[i]);
  double Q = kHankelAsym.q[7];
#pragma unroll
  for (int i = 6; i >= 0; --i) Q = fma(Q, w2, kHankelAsym.q[i]);
  Q *= w;
  // H0 = sqrt(2/(pi z)) e^{i(z - pi/4)} (P + i Q)
  double s, c;
  sincos(z, &s, &c);
  const double cw = (c + s) * 0.70710678118654752;   // cos(z - pi/4)
  const double sw = (s - c) * 0.70710678118654752;   // sin(z - pi/4)
  const double amp = sqrt(0.63661977236758134 * w);  // sqrt(2/(pi z))
  J = amp * (P * cw - Q * sw);
  Y = amp * (P * sw + Q * cw);
}

__device__ __forceinline__ void bessel01_series(double z, double& J, double& Y) {
  // J0 = sum (-1)^k u^k/(k!)^2, Y0 = (2/pi)(ln(z/2)+gamma) J0 + (2/pi) sum (-1)^{k+1} H_k u^k/(k!)^2,
  // u = z^2/4 (z < 2 so u < 1, no cancellation).
  const double u = 0.25 * z * z;
  double term = 1.0, Jsum = 1.0, S = 0.0, H = 0.0;
#pragma unroll
  for (int k = 1; k <= 20; ++k) {
    term *= -u * (1.0 / (double)(k * k));
    H += 1.0 / (double)k;  // literal after unrolling
    Jsum += term;
    S -= term * H;
  }
  J = Jsum;
  Y = 0.63661977236758134 * ((log(0.5 * z) + 0.57721566490153286) * Jsum + S);
}

// Miller's algorithm on 2 <= z < 25: backward recurrence J_{k-1} = (2k/z) J_k - J_{k+1} from the
// fixed even start order 56 (>= z + 30, enough for 1e-15), normalised with
// 1 = J0 + 2 sum_{k>=1} J_2k; Neumann's series gives
// Y0 = (2/pi)(ln(z/2) + gamma) J0 - (4/pi) sum_{k>=1} (-1)^k J_2k / k.
// The loop is fully unrolled so that every 1/k is a literal.
__device__ __forceinline__ void bessel01_miller(double z, double& J, double& Y) {
  constexpr int M = 56;
  const double two_over_z = 2.0 / z;
  double jp1 = 0.0, j = 1e-250;  // J_{M+1}, J_M up to a common scale
  double norm = 2.0 * j;
  double neu = ((M / 2) % 2 ? -j : j) * (1.0 / (M / 2));
#pragma unroll
  for (int k = M; k > 0; --k) {
    const double jm1 = fma((double)k * two_over_z, j, -jp1);  // J_{k-1}
    jp1 = j;
    j = jm1;
    const int e = k - 1;
    if (e > 0 && (e % 2) == 0) {
      const int h = e / 2;
      norm += 2.0 * j;
      neu += ((h % 2) ? -j : j) * (1.0 / h);
    }
  }
  norm += j;  // + J_0
  const double inv = 1.0 / norm;
  J = j * inv;
  Y = 0.63661977236758134 * (log(0.5 * z) + 0.57721566490153286) * J - 1.2732395447351627 * neu * inv;
}

// (i/4) H0^(1)(kappa r) from r (FP64).
__device__ __forceinline__ void phi2d_f64(double r, double kappa, double& pr, double& pi) {
  const double z = kappa * r;
  double J, Y;
  if (z >= 25.0) {
    hankel0_asym(z, J, Y);
  } else if (z >= 2.0) {
    bessel01_miller(z, J, Y);
  } else {
    bessel01_series(z, J, Y);
  }
  pr = -0.25 * Y;
  pi = 0.25 * J;
}

__device__ __forceinline__ void phi3d_f64(double r, double kappa, double& pr, double& pi) {
  double s, c;
  sincos(kappa * r, &s, &c);
  const double a = 0.079577471545947668 / r;
  pr = a * c;
  pi = a * s;
}

}  // namespace mfs
