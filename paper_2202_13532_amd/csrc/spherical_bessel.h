// Spherical Bessel function of the first kind j_s(z) for real z, shared by
// the host setup of the connection tensor and the device-side table builder
// of the allocation-free entry point (eq. spectral_transform).
//   |z| <= 8: ascending power series
//     j_s(z) = z^s / (2s+1)!! sum_k (-z^2/2)^k / (k! (2s+3)(2s+5)...(2s+2k+1));
//   beyond: Miller's downward recurrence j_{k-1} = (2k+1)/z j_k - j_{k+1},
//     normalised by j_0 = sin z / z or j_1 = sin z / z^2 - cos z / z.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace dgh {

__host__ __device__ inline double sph_bessel_j(int s, double z) {
  double sign = 1.0;
  if (z < 0.0) {
    z = -z;
    if (s % 2) sign = -1.0;
  }
  if (z == 0.0) return s == 0 ? 1.0 : 0.0;
  if (z <= 8.0) {
    double term = 1.0;
    for (int k = 1; k <= s; ++k) term *= z / (2.0 * k + 1.0);
    double sum = term;
    const double h = -0.5 * z * z;
    for (int k = 1; k < 200; ++k) {
      term *= h / (k * (2.0 * s + 2.0 * k + 1.0));
      sum += term;
      if (fabs(term) < 1e-18 * fabs(sum)) break;
    }
    return sign * sum;
  }
  const int top = s + 30 + static_cast<int>(z);
  double jp1 = 0.0, j = 1e-250, js = 0.0, j0 = 0.0, j1 = 0.0;
  for (int k = top; k >= 1; --k) {
    const double jm1 = (2.0 * k + 1.0) / z * j - jp1;
    jp1 = j;
    j = jm1;
    if (k - 1 == s) js = j;
    if (k - 1 == 1) j1 = j;
    if (k - 1 == 0) j0 = j;
    if (fabs(j) > 1e200) {  // rescale to stay in range
      j *= 1e-200;
      jp1 *= 1e-200;
      js *= 1e-200;
      j1 *= 1e-200;
    }
  }
  const double t0 = sin(z) / z, t1 = sin(z) / (z * z) - cos(z) / z;
  return sign * (fabs(t0) > fabs(t1) ? js * (t0 / j0) : js * (t1 / j1));
}

}  // namespace dgh
