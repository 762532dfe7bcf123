// Device-side helpers shared by the kernel translation units of libmbstokes (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace mbs {

constexpr double RS2 = 0.70710678118654752440;  // 1/sqrt(2)
constexpr double RS6 = 0.40824829046386301637;  // 1/sqrt(6)
constexpr int kMaxBlock = 256;

// 1/sqrt(r2) for r2 > 0.
// binary64: hardware reciprocal square root estimate followed by one Newton-Raphson step
// y <- y + (y/2)(1 - r2 y^2), which squares the relative error of the estimate.
__device__ __forceinline__ double rsq_nr(double r2) {
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2 * y0, y0, 1.0);
  return fma(0.5 * y0, e, y0);
}
// binary32: the hardware estimate (about 1 ulp).
__device__ __forceinline__ float rsq_nr(float r2) { return __builtin_amdgcn_rsqf(r2); }

// Same, but 0 for r2 == 0 (the n == m term), without a branch.
__device__ __forceinline__ double rinv_or_zero(double r2) {
  const double y = rsq_nr(r2);
  return r2 > 0.0 ? y : 0.0;
}
__device__ __forceinline__ float rinv_or_zero(float r2) {
  const float y = rsq_nr(r2);
  return r2 > 0.0f ? y : 0.0f;
}

// Accumulate sym(x (x) v) in the 5-basis scaled by (sqrt2, sqrt6, sqrt2, sqrt2, sqrt2).
template <typename T>
__device__ __forceinline__ void acc_sym(T dx, T dy, T dz, T vx, T vy, T vz, T& a0, T& a1, T& a2,
                                        T& a3, T& a4) {
  const T pxx = dx * vx, pyy = dy * vy, pzz = dz * vz;
  a0 += pxx - pyy;
  a1 += (T)2 * pzz - pxx - pyy;
  a2 += dx * vy + dy * vx;
  a3 += dx * vz + dz * vx;
  a4 += dy * vz + dz * vy;
}

// Cartesian components of a symmetric traceless tensor from its 5-basis coefficients
// (Szz = -Sxx - Syy).
__device__ __forceinline__ void basis_to_cart(const double* s, double& sxx, double& syy,
                                              double& sxy, double& sxz, double& syz) {
  const double u0 = s[0] * RS2, u1 = s[1] * RS6;
  sxx = u0 - u1;
  syy = -u0 - u1;
  sxy = s[2] * RS2;
  sxz = s[3] * RS2;
  syz = s[4] * RS2;
}

}  // namespace mbs
