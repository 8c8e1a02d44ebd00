// FP64 host construction of the LGL -> Fourier connection tensor (Sec. 5.3,
// eq. spectral_transform).
#include <cmath>
#include <complex>
#include <vector>

#include "dg_host.h"
#include "spherical_bessel.h"

namespace dgh {

using cd = std::complex<double>;

double spherical_bessel_j(int s, double z) { return sph_bessel_j(s, z); }

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
