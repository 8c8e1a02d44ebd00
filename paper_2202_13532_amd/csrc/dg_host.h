// Host-side FP64 setup of the DG operators and the spectral Poisson tables.
#pragma once
#include <complex>
#include <vector>

namespace dgh {

// Reference-element LGL operators (Sec. 5.2).  Matrices are row-major with the
// output node first: (ups * F)_i = sum_k ups[i*n + k] F_k.
struct Basis {
  int n = 0;
  std::vector<double> xi, w;      // nodes (ascending), weights
  std::vector<double> dmat;       // D[j*n + k] = l'_k(xi_j)
  std::vector<double> ups;        // Upsilon (eq. num_flux_wow)
  std::vector<double> xi_face;    // Xi[i*2 + c], c = 0 left face, 1 right face
  std::vector<double> pn;         // P_{n-1}(xi_j)
};

double legendre(int s, double x);
double legendre_deriv(int s, double x);
Basis make_basis(int n);

// Spherical Bessel function of the first kind j_s(z), real z.
double spherical_bessel_j(int s, double z);

// Connection tensor T_p^{mj} (eq. spectral_transform) for p = 1..pmax on an
// axis of nelem equal elements spanning [lo, hi]: index ((p-1)*nelem + m)*n + j.
std::vector<std::complex<double>> connection_tensor(const Basis& b, int nelem, double lo,
                                                    double hi, int pmax);

// Eigenvalues of a small complex matrix (row-major, m x m).
std::vector<std::complex<double>> eigenvalues(std::vector<std::complex<double>> a, int m);

// RK3 + upwind weak-DG Courant number C_n: dt <= C_n dx / |a| is stable.
double courant_number(int n);

}  // namespace dgh
