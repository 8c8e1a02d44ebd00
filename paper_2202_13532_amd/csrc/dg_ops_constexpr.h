// Compile-time LGL reference operators for the device kernels.
//
// The stage kernels are specialised on the node count n; evaluating the
// operators at compile time turns every matrix entry into an instruction
// literal, so the contractions need no registers for them.  The formulas are
// those of Sec. 5.2: nodes = zeros of (1 - xi^2) P'_{n-1}, weights
// (eq. quad_weights), Lagrange derivative D_jk = l'_k(xi_j), and
//   Upsilon^j_k = (w_k / w_j) l'_j(xi_k) + (n/2) w_k P_{n-1}(xi_j) P'_{n-1}(xi_k),
//   Xi^j_c      = delta_{j, end c} / w_j + (n/2) P_{n-1}(xi_j) P_{n-1}(xi_{end c})
// (eq. num_flux_wow).  The host FP64 setup in basis.cpp computes the same
// quantities at run time for the tables and the introspection calls.
#pragma once

namespace dgc {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double c_cos(double x) {  // Taylor series, |x| <= pi
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr double c_leg(int s, double x) {
  if (s == 0) return 1.0;
  double pm = 1.0, p = x;
  for (int k = 1; k < s; ++k) {
    const double pn = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
    pm = p;
    p = pn;
  }
  return p;
}

constexpr double c_dleg(int s, double x) {
  if (s == 0) return 0.0;
  if (x == 1.0) return 0.5 * s * (s + 1.0);
  if (x == -1.0) return ((s + 1) % 2 ? -1.0 : 1.0) * 0.5 * s * (s + 1.0);
  return s * (c_leg(s - 1, x) - x * c_leg(s, x)) / (1.0 - x * x);
}

template <int N>
struct OpsC {
  double xi[N] = {};
  double w[N] = {};
  double ups[N][N] = {};
  double xl[N] = {};
  double xr[N] = {};
};

template <int N>
constexpr OpsC<N> make_ops() {
  OpsC<N> o{};
  const int M = N - 1;
  o.xi[0] = -1.0;
  o.xi[M] = 1.0;
  for (int j = 1; j < M; ++j) {
    double t = -c_cos(kPi * j / M);
    for (int it = 0; it < 60; ++it) {
      const double p = c_leg(M, t), dp = c_dleg(M, t);
      const double d2p = (2.0 * t * dp - M * (M + 1.0) * p) / (1.0 - t * t);
      if (d2p == 0.0) break;
      t -= dp / d2p;
    }
    o.xi[j] = t;
  }
  for (int j = 0; j < N / 2; ++j) {
    const double s = 0.5 * (o.xi[M - j] - o.xi[j]);
    o.xi[j] = -s;
    o.xi[M - j] = s;
  }
  if (N % 2) o.xi[M / 2] = 0.0;
  double pn[N] = {};
  for (int j = 0; j < N; ++j) {
    pn[j] = c_leg(M, o.xi[j]);
    o.w[j] = 2.0 / (N * (N - 1.0) * pn[j] * pn[j]);
  }
  double D[N][N] = {};
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      if (j != k) D[j][k] = pn[j] / (pn[k] * (o.xi[j] - o.xi[k]));
  D[0][0] = -0.25 * M * (M + 1.0);
  D[M][M] = 0.25 * M * (M + 1.0);
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < N; ++k)
      o.ups[j][k] = (o.w[k] / o.w[j]) * D[k][j] + 0.5 * N * o.w[k] * pn[j] * c_dleg(M, o.xi[k]);
  for (int j = 0; j < N; ++j) {
    o.xl[j] = (j == 0 ? 1.0 / o.w[j] : 0.0) + 0.5 * N * pn[j] * pn[0];
    o.xr[j] = (j == M ? 1.0 / o.w[j] : 0.0) + 0.5 * N * pn[j] * pn[M];
  }
  return o;
}

// The even/odd contraction relies on Ups[n-1-i][n-1-k] = -Ups[i][k] and
// Xr[i] = Xl[n-1-i] (reflection symmetry of the LGL node set).
template <int N>
constexpr bool reflection_symmetric() {
  const OpsC<N> o = make_ops<N>();
  double scale = 1.0;
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k) scale = o.ups[i][k] > scale ? o.ups[i][k] : (-o.ups[i][k] > scale ? -o.ups[i][k] : scale);
  for (int i = 0; i < N; ++i) {
    const double dx = o.xr[i] - o.xl[N - 1 - i];
    if ((dx < 0 ? -dx : dx) > 1e-12 * scale) return false;
    for (int k = 0; k < N; ++k) {
      const double d = o.ups[N - 1 - i][N - 1 - k] + o.ups[i][k];
      if ((d < 0 ? -d : d) > 1e-12 * scale) return false;
    }
  }
  return true;
}

}  // namespace dgc
