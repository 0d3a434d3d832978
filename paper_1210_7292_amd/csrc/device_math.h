// Device helpers shared by the uniform and adaptive passes: the 1-D Chebyshev interpolation
// basis of Sec. 2.1 and its derivative, and the kernel functions with their radial derivative.
#pragma once

#include <hip/hip_runtime.h>

#include "host_math.h"

namespace bbfmm {

// S_l(u, xbar_m) = 1/l + 2/l sum_{k>=1} T_k(u) T_k(xbar_m) for all m; tk[k*L + m] = T_k(xbar_m).
template <int L>
__device__ inline void cheb_basis_all(double u, const double* tk, double* out) {
  double t[L];
  t[0] = 1.0;
  if (L > 1) t[1] = u;
#pragma unroll
  for (int k = 2; k < L; ++k) t[k] = 2.0 * u * t[k - 1] - t[k - 2];
#pragma unroll
  for (int m = 0; m < L; ++m) {
    double s = 0.0;
#pragma unroll
    for (int k = 1; k < L; ++k) s += t[k] * tk[k * L + m];
    out[m] = (1.0 + 2.0 * s) / L;
  }
}

// d/du of the same basis: T_k'(u) = k U_{k-1}(u).
template <int L>
__device__ inline void cheb_basis_deriv_all(double u, const double* tk, double* out) {
  double uu[L > 1 ? L - 1 : 1];
  uu[0] = 1.0;
  if (L > 2) uu[1] = 2.0 * u;
#pragma unroll
  for (int k = 2; k < L - 1; ++k) uu[k] = 2.0 * u * uu[k - 1] - uu[k - 2];
#pragma unroll
  for (int m = 0; m < L; ++m) {
    double s = 0.0;
#pragma unroll
    for (int k = 1; k < L; ++k) s += k * uu[k - 1] * tk[k * L + m];
    out[m] = 2.0 * s / L;
  }
}

// The kernel's parameter as kern / kern_dr take it: c^2 for 1/sqrt(r^2 + c^2), the wavenumber k
// for the Helmholtz parts.
template <int KIND>
__host__ __device__ inline double kernel_param(double c) {
  return KIND == kInvSqrtR2C2 ? c * c : c;
}

template <int KIND>
__device__ inline double kern(double r2, double kp) {
  if (KIND == kInvR) {
    // branch-free: the select for r = 0 discards rsqrt(0) = inf
    const double ir = rsqrt(r2);
    return r2 > 0.0 ? ir : 0.0;
  }
  if (KIND == kInvSqrtR2C2) return rsqrt(r2 + kp);
  if (KIND == kHelmCos || KIND == kHelmSin) {
    // cos(kr)/r (0 at r = 0) and sin(kr)/r (k at r = 0): the parts of e^{ikr}/r
    if (!(r2 > 0.0)) return KIND == kHelmSin ? kp : 0.0;
    const double r = sqrt(r2);
    double sn, cs;
    sincos(kp * r, &sn, &cs);
    return (KIND == kHelmCos ? cs : sn) / r;
  }
  if (KIND == kR2) return r2;
  return r2 * r2;
}

// (1/r) dK/dr, so that grad_x K(x, y) = kern_dr(r2) * (x - y).
template <int KIND>
__device__ inline double kern_dr(double r2, double kp) {
  if (KIND == kInvR) {
    const double ir = rsqrt(r2);
    return r2 > 0.0 ? -ir * ir * ir : 0.0;
  }
  if (KIND == kInvSqrtR2C2) {
    const double ir = rsqrt(r2 + kp);
    return -ir * ir * ir;
  }
  if (KIND == kHelmCos || KIND == kHelmSin) {
    const double r = sqrt(r2), kr = kp * r;
    if (KIND == kHelmSin && kr < 0.05) {
      // (k r cos(kr) - sin(kr)) / r^3 cancels for small kr: its Taylor series
      const double k2 = kp * kp;
      return kp * k2 * (-1.0 / 3.0 + k2 * r2 * (1.0 / 30.0 - k2 * r2 / 840.0));
    }
    if (!(r2 > 0.0)) return 0.0;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double ir3 = 1.0 / (r2 * r);
    return (KIND == kHelmCos ? -(kr * sn + cs) : (kr * cs - sn)) * ir3;
  }
  if (KIND == kR2) return 2.0;
  return 4.0 * r2;
}

}  // namespace bbfmm
