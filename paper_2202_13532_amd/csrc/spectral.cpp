// FP64 host construction of the LGL -> Fourier connection tensor (Sec. 5.3,
// eq. spectral_transform).
#include <cmath>
#include <complex>
#include <vector>

#include "dg_host.h"

namespace dgh {

using cd = std::complex<double>;

// j_s(z): ascending power series for |z| <= 8,
//   j_s(z) = z^s / (2s+1)!! sum_k (-z^2/2)^k / (k! (2s+3)(2s+5)...(2s+2k+1)),
// and Miller's downward recurrence j_{k-1} = (2k+1)/z j_k - j_{k+1},
// normalised by j_0 = sin z / z or j_1 = sin z / z^2 - cos z / z, beyond.
double spherical_bessel_j(int s, double z) {
  if (z < 0.0) return ((s % 2) ? -1.0 : 1.0) * spherical_bessel_j(s, -z);
  if (z == 0.0) return s == 0 ? 1.0 : 0.0;
  if (z <= 8.0) {
    double term = 1.0;
    for (int k = 1; k <= s; ++k) term *= z / (2.0 * k + 1.0);
    double sum = term;
    const double h = -0.5 * z * z;
    for (int k = 1; k < 200; ++k) {
      term *= h / (k * (2.0 * s + 2.0 * k + 1.0));
      sum += term;
      if (std::fabs(term) < 1e-18 * std::fabs(sum)) break;
    }
    return sum;
  }
  const int top = s + 30 + static_cast<int>(z);
  double jp1 = 0.0, j = 1e-250, js = 0.0, j0 = 0.0, j1 = 0.0;
  for (int k = top; k >= 1; --k) {
    double jm1 = (2.0 * k + 1.0) / z * j - jp1;
    jp1 = j;
    j = jm1;
    if (k - 1 == s) js = j;
    if (k - 1 == 1) j1 = j;
    if (k - 1 == 0) j0 = j;
    if (std::fabs(j) > 1e200) {  // rescale to stay in range
      j *= 1e-200; jp1 *= 1e-200; js *= 1e-200; j1 *= 1e-200;
    }
  }
  double t0 = std::sin(z) / z, t1 = std::sin(z) / (z * z) - std::cos(z) / z;
  return std::fabs(t0) > std::fabs(t1) ? js * (t0 / j0) : js * (t1 / j1);
}

std::vector<cd> connection_tensor(const Basis& b, int nelem, double lo, double hi, int pmax) {
  const int n = b.n;
  const double L = hi - lo, dx = L / nelem, J = 2.0 / dx;
  std::vector<double> gamma(n);
  for (int s = 0; s < n; ++s) gamma[s] = (s < n - 1) ? 2.0 / (2.0 * s + 1.0) : 2.0 / (n - 1.0);
  std::vector<cd> mi(n);  // (-i)^s
  for (int s = 0; s < n; ++s) {
    static const cd pw[4] = {cd(1, 0), cd(0, -1), cd(-1, 0), cd(0, 1)};
    mi[s] = pw[s % 4];
  }
  std::vector<cd> out(static_cast<size_t>(pmax) * nelem * n);
  for (int p = 1; p <= pmax; ++p) {
    const double kp = 2.0 * M_PI * p / L;
    // tau_p^j = w_j sum_s gamma_s^-1 (-i)^s P_s(xi_j) j_s(k_p / J): identical
    // for every element of equal width (Sec. 5.3.1), times dx/L e^{-i k_p xbar_m}.
    std::vector<cd> tau(n);
    for (int j = 0; j < n; ++j) {
      cd acc = 0.0;
      for (int s = 0; s < n; ++s)
        acc += mi[s] * (legendre(s, b.xi[j]) * spherical_bessel_j(s, kp / J) / gamma[s]);
      tau[j] = b.w[j] * acc;
    }
    for (int m = 0; m < nelem; ++m) {
      const double xbar = lo + (m + 0.5) * dx;
      const cd ph = (dx / L) * std::polar(1.0, -kp * xbar);
      for (int j = 0; j < n; ++j) out[(static_cast<size_t>(p - 1) * nelem + m) * n + j] = ph * tau[j];
    }
  }
  return out;
}

}  // namespace dgh
