// FP64 host construction of the LGL reference operators and the RK3 stability
// limit.  Formulas follow Sec. 5.2 of the paper (eq. quad_weights, eq. minv,
// eq. num_flux_wow); the derivative matrix uses the classical closed form of
// the Lagrange derivative on Lobatto nodes.
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

#include "dg_host.h"

namespace dgh {

using cd = std::complex<double>;

double legendre(int s, double x) {
  if (s == 0) return 1.0;
  double pm = 1.0, p = x;
  for (int k = 1; k < s; ++k) {
    double pn = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
    pm = p;
    p = pn;
  }
  return p;
}

// P'_s(x); at x = +-1 uses P'_s(+-1) = (+-1)^(s+1) s (s+1) / 2.
double legendre_deriv(int s, double x) {
  if (s == 0) return 0.0;
  if (x == 1.0) return 0.5 * s * (s + 1.0);
  if (x == -1.0) return ((s + 1) % 2 ? -1.0 : 1.0) * 0.5 * s * (s + 1.0);
  // (1 - x^2) P'_s = s (P_{s-1} - x P_s)
  return s * (legendre(s - 1, x) - x * legendre(s, x)) / (1.0 - x * x);
}

// Interior LGL nodes are the zeros of P'_N (N = n - 1).  Newton's method on
// P'_N with P''_N from the Legendre equation (1 - x^2) P'' = 2 x P' - N(N+1) P.
static std::vector<double> lgl_nodes(int n) {
  const int N = n - 1;
  std::vector<double> x(n);
  x[0] = -1.0;
  x[N] = 1.0;
  for (int j = 1; j < N; ++j) {
    double t = -std::cos(M_PI * j / N);
    for (int it = 0; it < 100; ++it) {
      double p = legendre(N, t), dp = legendre_deriv(N, t);
      double d2p = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
      double step = dp / d2p;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[j] = t;
  }
  for (int j = 0; j < n / 2; ++j) {  // enforce the exact symmetry of the rule
    double s = 0.5 * (x[N - j] - x[j]);
    x[j] = -s;
    x[N - j] = s;
  }
  if (n % 2) x[N / 2] = 0.0;
  return x;
}

Basis make_basis(int n) {
  if (n < 2) throw std::invalid_argument("n < 2");
  const int N = n - 1;
  Basis b;
  b.n = n;
  b.xi = lgl_nodes(n);
  b.w.resize(n);
  b.pn.resize(n);
  for (int j = 0; j < n; ++j) {
    b.pn[j] = legendre(N, b.xi[j]);
    b.w[j] = 2.0 / (n * (n - 1.0) * b.pn[j] * b.pn[j]);  // eq. quad_weights
  }
  // D_jk = l'_k(xi_j): P_N(xi_j) / (P_N(xi_k) (xi_j - xi_k)) off the diagonal,
  // -N(N+1)/4 and +N(N+1)/4 at the two end points, 0 elsewhere on the diagonal.
  b.dmat.assign(n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (j != k) b.dmat[j * n + k] = b.pn[j] / (b.pn[k] * (b.xi[j] - b.xi[k]));
  b.dmat[0] = -0.25 * N * (N + 1.0);
  b.dmat[N * n + N] = 0.25 * N * (N + 1.0);
  // eq. num_flux_wow:
  //   Upsilon^j_k = (w_k / w_j) l'_j(xi_k) + (n/2) w_k P_N(xi_j) P'_N(xi_k)
  //   Xi^j_c      = delta_{j, end c} / w_j + (n/2) P_N(xi_j) P_N(xi_{end c})
  b.ups.assign(n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      double dpk = legendre_deriv(N, b.xi[k]);
      b.ups[j * n + k] = (b.w[k] / b.w[j]) * b.dmat[k * n + j] + 0.5 * n * b.w[k] * b.pn[j] * dpk;
    }
  b.xi_face.assign(n * 2, 0.0);
  for (int j = 0; j < n; ++j) {
    b.xi_face[j * 2 + 0] = (j == 0 ? 1.0 / b.w[j] : 0.0) + 0.5 * n * b.pn[j] * b.pn[0];
    b.xi_face[j * 2 + 1] = (j == N ? 1.0 / b.w[j] : 0.0) + 0.5 * n * b.pn[j] * b.pn[N];
  }
  return b;
}

// Eigenvalues by Householder reduction to Hessenberg form followed by a
// Wilkinson-shifted complex QR iteration with Givens rotations.
std::vector<cd> eigenvalues(std::vector<cd> a, int m) {
  auto A = [&](int i, int j) -> cd& { return a[i * m + j]; };
  for (int k = 0; k + 2 < m; ++k) {
    double nrm = 0.0;
    for (int i = k + 1; i < m; ++i) nrm += std::norm(A(i, k));
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    cd x0 = A(k + 1, k);
    cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
    cd alpha = -ph * nrm;
    std::vector<cd> v(m, 0.0);
    for (int i = k + 1; i < m; ++i) v[i] = A(i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < m; ++i) v[i] /= vn;
    for (int j = 0; j < m; ++j) {  // A <- (I - 2 v v^H) A
      cd s = 0.0;
      for (int i = k + 1; i < m; ++i) s += std::conj(v[i]) * A(i, j);
      for (int i = k + 1; i < m; ++i) A(i, j) -= 2.0 * v[i] * s;
    }
    for (int i = 0; i < m; ++i) {  // A <- A (I - 2 v v^H)
      cd s = 0.0;
      for (int j = k + 1; j < m; ++j) s += A(i, j) * v[j];
      for (int j = k + 1; j < m; ++j) A(i, j) -= 2.0 * s * std::conj(v[j]);
    }
  }
  std::vector<cd> eig;
  int hi = m - 1, iter = 0;
  const double eps = 1e-15;
  std::vector<cd> gc(m), gs(m);
  while (hi > 0) {
    int l = hi;
    while (l > 0 && std::abs(A(l, l - 1)) > eps * (std::abs(A(l, l)) + std::abs(A(l - 1, l - 1)) + 1e-300)) --l;
    if (l == hi) {
      eig.push_back(A(hi, hi));
      --hi;
      iter = 0;
      continue;
    }
    if (iter > 500) throw std::runtime_error("QR did not converge");
    cd a11 = A(hi - 1, hi - 1), a12 = A(hi - 1, hi), a21 = A(hi, hi - 1), a22 = A(hi, hi);
    cd tr = a11 + a22, det = a11 * a22 - a12 * a21;
    cd disc = std::sqrt(tr * tr / 4.0 - det);
    cd mu1 = tr / 2.0 + disc, mu2 = tr / 2.0 - disc;
    cd mu = std::abs(mu1 - a22) < std::abs(mu2 - a22) ? mu1 : mu2;
    if (iter % 11 == 10) mu = a22 + std::abs(a21);
    for (int i = l; i <= hi; ++i) A(i, i) -= mu;
    for (int k = l; k < hi; ++k) {
      cd x = A(k, k), y = A(k + 1, k);
      double r = std::sqrt(std::norm(x) + std::norm(y));
      cd c = r > 0 ? x / r : cd(1.0, 0.0), s = r > 0 ? y / r : cd(0.0, 0.0);
      gc[k] = c;
      gs[k] = s;
      for (int j = k; j <= hi; ++j) {
        cd p = A(k, j), q = A(k + 1, j);
        A(k, j) = std::conj(c) * p + std::conj(s) * q;
        A(k + 1, j) = -s * p + c * q;
      }
    }
    for (int k = l; k < hi; ++k) {
      cd c = gc[k], s = gs[k];
      int rmax = std::min(k + 2, hi);
      for (int i = l; i <= rmax; ++i) {
        cd p = A(i, k), q = A(i, k + 1);
        A(i, k) = p * c + q * s;
        A(i, k + 1) = -p * std::conj(s) + q * std::conj(c);
      }
    }
    for (int i = l; i <= hi; ++i) A(i, i) += mu;
    ++iter;
  }
  eig.push_back(A(0, 0));
  return eig;
}

// For u_t + u_x = 0 with periodic identical elements, the Bloch mode
// u_{m+1} = e^{i theta} u_m gives the one-element operator (J = 1)
//   L(theta) = Upsilon + e^{-i theta} Xi_left e_last^T - Xi_right e_last^T.
// dt lambda must lie in the RK3 region |1 + z + z^2/2 + z^3/6| <= 1; with
// J = 2/dx, z = 2 C lambda for dt = C dx.  C_n is found by bisection.
double courant_number(int n) {
  Basis b = make_basis(n);
  std::vector<cd> lam;
  const int nth = 1024;
  for (int t = 0; t <= nth; ++t) {
    double th = 2.0 * M_PI * t / nth;
    cd e = std::polar(1.0, -th);
    std::vector<cd> L(n * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        cd v = b.ups[i * n + k];
        if (k == n - 1) v += e * b.xi_face[i * 2 + 0] - b.xi_face[i * 2 + 1];
        L[i * n + k] = v;
      }
    auto ev = eigenvalues(L, n);
    lam.insert(lam.end(), ev.begin(), ev.end());
  }
  double lo = 0.0, hi = 2.0;
  for (int it = 0; it < 60; ++it) {
    double c = 0.5 * (lo + hi);
    double worst = 0.0;
    for (const cd& l : lam) {
      cd z = 2.0 * c * l;
      worst = std::max(worst, std::abs(1.0 + z + z * z / 2.0 + z * z * z / 6.0));
    }
    if (worst <= 1.0 + 1e-12) lo = c; else hi = c;
  }
  return lo;
}

}  // namespace dgh
