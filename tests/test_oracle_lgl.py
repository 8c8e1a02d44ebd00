"""Pins of oracle.lgl against textbook values, library routines and quadrature."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import lgl
from tests.golden import paper_value


def test_textbook_node_sets():
    # n = 3: {-1, 0, 1}, weights {1/3, 4/3, 1/3} (stored with its citation)
    x, w = lgl.lgl_nodes_weights(3)
    g = paper_value("lgl_n3")
    assert np.allclose(x, g["nodes"], atol=1e-15)
    assert np.allclose(w, g["weights"], atol=1e-15)
    # n = 4: {+-1, +-1/sqrt5}, weights {1/6, 5/6}
    x, w = lgl.lgl_nodes_weights(4)
    s = 1 / math.sqrt(5)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)
    # n = 5: {0, +-sqrt(3/7), +-1}, weights {32/45, 49/90, 1/10}
    x, w = lgl.lgl_nodes_weights(5)
    r = math.sqrt(3 / 7)
    assert np.allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("n", range(3, 13))
def test_interior_nodes_are_jacobi_roots(n):
    # zeros of P'_{n-1} are the zeros of the Jacobi polynomial P^{(1,1)}_{n-2}
    x, _ = lgl.lgl_nodes_weights(n)
    roots, _ = sp.roots_jacobi(n - 2, 1.0, 1.0)
    assert np.allclose(np.sort(roots), x[1:-1], atol=1e-14)


@pytest.mark.parametrize("n", range(2, 13))
def test_quadrature_exact_to_degree_2n_minus_3(n):
    x, w = lgl.lgl_nodes_weights(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * n - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13, (n, k)
    # not exact one degree higher (even degree 2n-2)
    k = 2 * n - 2
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-9


@pytest.mark.parametrize("n", range(2, 13))
def test_derivative_matrix_exact_on_polynomials(n):
    rng = np.random.default_rng(n)
    x, _ = lgl.lgl_nodes_weights(n)
    D = lgl.derivative_matrix(x)
    for _ in range(3):
        c = rng.standard_normal(n)        # degree n-1
        p = np.polynomial.Polynomial(c)
        assert np.max(np.abs(D @ p(x) - p.deriv()(x))) < 1e-11 * max(1, np.abs(c).sum() * n * n)


def _brute_integrals(n):
    x, _ = lgl.lgl_nodes_weights(n)
    eta, om = np.polynomial.legendre.leggauss(n + 6)
    L = np.stack([lgl.lagrange_eval(x, j, eta) for j in range(n)])
    h = 1e-6
    # derivative of the basis by exact differentiation of the interpolating polynomial
    dL = np.stack([np.polynomial.Polynomial.fit(x, np.eye(n)[j], n - 1).deriv()(eta) for j in range(n)])
    M = (L * om) @ L.T
    S = (dL * om) @ L.T          # S_ij = int l_i' l_j
    return M, S


@pytest.mark.parametrize("n", range(2, 13))
def test_operators_against_quadrature(n):
    o = lgl.operators(n)
    M, S = _brute_integrals(n)
    assert np.allclose(M @ o["Minv"], np.eye(n), atol=1e-11)
    assert np.allclose(o["S"], S, atol=1e-10)
    Minv_b = np.linalg.inv(M)
    assert np.allclose(o["Ups"], Minv_b @ S, atol=1e-9 * n * n)
    assert np.allclose(o["Xi"][:, 0], Minv_b[:, 0], atol=1e-9 * n * n)
    assert np.allclose(o["Xi"][:, 1], Minv_b[:, -1], atol=1e-9 * n * n)


@pytest.mark.parametrize("n", range(2, 13))
def test_paper_closed_forms(n):
    """M^-1 S agrees with eq. num_flux_wow, eq. internal_flux_wow, eq. derivative."""
    o = lgl.operators(n)
    x, w, D = o["xi"], o["w"], o["D"]
    P = lgl.legendre(n - 1, x)
    dP = lgl.legendre_deriv(n - 1, x)
    gamma = np.array([2.0 / (2 * s + 1) for s in range(n - 1)] + [2.0 / (n - 1)])
    # Upsilon^j_k = (w_k/w_j) l_j'(xi_k) + (n/2) w_k P(xi_j) P'(xi_k)
    ups1 = (w[None, :] / w[:, None]) * D.T + 0.5 * n * np.outer(P, w * dP)
    # Upsilon^j_k = w_k sum_s (s + 1/2) P_s(xi_j) P_s'(xi_k)
    ups2 = sum((s + 0.5) * np.outer(lgl.legendre(s, x), w * lgl.legendre_deriv(s, x)) for s in range(n))
    # D^j_k = w_k sum_s P_s'(xi_j) P_s(xi_k) / gamma_s
    D2 = sum(np.outer(lgl.legendre_deriv(s, x), w * lgl.legendre(s, x)) / gamma[s] for s in range(n))
    tol = 1e-11 * n ** 3
    assert np.allclose(o["Ups"], ups1, atol=tol)
    assert np.allclose(o["Ups"], ups2, atol=tol)
    assert np.allclose(D, D2, atol=tol)
    # eq. cool_identity: sum_s P_{n-1}(xi_s) l_s'(xi_j) = P'_{n-1}(xi_j)
    assert np.allclose(D @ P, dP, atol=tol)
    # discrete orthogonality with the Lobatto-weighted last eigenvalue (eq. discrete_orthogonality)
    V = np.stack([lgl.legendre(s, x) for s in range(n)], axis=1)
    assert np.allclose((V.T * w) @ V, np.diag(gamma), atol=1e-12)
    # mass matrix as diagonal minus rank one
    alpha = n * (n - 1) / (2.0 * (2 * n - 1))
    M = np.diag(w) - alpha * np.outer(w * P, w * P)
    assert np.allclose(M @ o["Minv"], np.eye(n), atol=1e-11)


@pytest.mark.parametrize("n", range(2, 13))
def test_summation_by_parts_and_mass_row(n):
    o = lgl.operators(n)
    B = np.zeros((n, n)); B[0, 0] = -1; B[-1, -1] = 1
    assert np.allclose(o["A"] + o["A"].T, B, atol=1e-12)
    # w^T M^-1 = 1^T (used by conservation)
    assert np.allclose(o["w"] @ o["Minv"], np.ones(n), atol=1e-11)
    # constants are in the kernel of the stiffness action: Upsilon 1 ... w^T Upsilon = 0 per column sums
    assert np.allclose(o["w"] @ o["Ups"], 0.0, atol=1e-11)
