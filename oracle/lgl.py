"""One-dimensional Legendre-Gauss-Lobatto (LGL) basis and DG operators, FP64.

Test infrastructure (see ``oracle/__init__``).

Follows Sec. 5.2 ("DG matrices in the Lobatto basis"):
  * nodes are the zeros of (1 - xi^2) P'_{n-1}(xi), weights
    w_j = 2 / (n (n-1) P_{n-1}(xi_j)^2)                       (eq. quad_weights)
  * inverse mass matrix  M^-1_ij = delta_ij / w_i + (n/2) P_{n-1}(xi_i) P_{n-1}(xi_j)
                                                             (eq. minv)
  * advection A_ij = w_i l'_j(xi_i) and stiffness S = A^T, S_ij = w_j l'_i(xi_j)
                                                             (eq. lobatto-advection)
  * weak-form internal flux operator Upsilon = M^-1 S, face operator
    Xi = first and last columns of M^-1, derivative D_jk = l'_k(xi_j)
                                                             (eq. num_flux_wow)
Matrices are stored with the OUTPUT node as the first index:
(Upsilon F)_i = sum_k Upsilon[i, k] F_k.

Pinned by tests/test_oracle_lgl.py against textbook node sets, quadrature
exactness, scipy's Jacobi roots, exact polynomial differentiation, brute-force
Gauss-Legendre integrals of the Lagrange basis, and the paper's alternative
closed forms (eq. internal_flux_wow, eq. derivative, eq. cool_identity).
"""
import numpy as np


def legendre(s, x):
    """P_s(x) by Bonnet's three-term recurrence (float64, any array x)."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if s == 0:
        return p_prev
    p = x.copy()
    for k in range(1, s):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p


def legendre_deriv(s, x):
    """P'_s(x) from the recurrence of derivatives P'_{k+1} = P'_{k-1} + (2k+1) P_k."""
    x = np.asarray(x, dtype=np.float64)
    if s == 0:
        return np.zeros_like(x)
    d_prev = np.zeros_like(x)        # P'_0
    d = np.ones_like(x)              # P'_1
    for k in range(1, s):
        d_prev, d = d, d_prev + (2 * k + 1) * legendre(k, x)
    return d


def lgl_nodes_weights(n):
    """LGL nodes (ascending) and weights for n >= 2 nodes (eq. quad_weights).

    The n nodes are the zeros of q(x) = (1 - x^2) P'_N(x), N = n - 1.  Using
    (1 - x^2) P'_N = N (P_{N-1} - x P_N) and the Legendre equation
    ((1 - x^2) P'_N)' = -N (N + 1) P_N, Newton's step for q is
        x <- x + (P_{N-1}(x) - x P_N(x)) / ((N + 1) P_N(x)),
    started from the Chebyshev-Gauss-Lobatto points -cos(pi j / N).
    """
    if n < 2:
        raise ValueError("LGL needs n >= 2")
    N = n - 1
    x = -np.cos(np.pi * np.arange(n) / N)
    for _ in range(100):
        pN = legendre(N, x)
        pNm1 = legendre(N - 1, x)
        dx = (pNm1 - x * pN) / ((N + 1) * pN)
        x = x + dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    # exact symmetry of the node set
    x = 0.5 * (x - x[::-1])
    w = 2.0 / (n * (n - 1) * legendre(N, x) ** 2)
    return x, w


def lagrange_eval(xi, j, x):
    """l_j(x) for the node set xi, by the product formula (eq. lagrange)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    for k in range(len(xi)):
        if k != j:
            out = out * (x - xi[k]) / (xi[j] - xi[k])
    return out


def derivative_matrix(xi):
    """D[j, k] = l'_k(xi_j) (eq. num_flux_wow, third line), barycentric form."""
    n = len(xi)
    lam = np.array([1.0 / np.prod([xi[j] - xi[k] for k in range(n) if k != j])
                    for j in range(n)])
    D = np.zeros((n, n))
    for j in range(n):
        for k in range(n):
            if j != k:
                D[j, k] = (lam[k] / lam[j]) / (xi[j] - xi[k])
        D[j, j] = -np.sum(D[j, :])
    return D


def mass_inverse(xi, w):
    """Closed-form inverse LGL mass matrix (eq. minv)."""
    n = len(xi)
    p = legendre(n - 1, xi)
    return np.diag(1.0 / w) + 0.5 * n * np.outer(p, p)


def stiffness(w, D):
    """S_ij = w_j l'_i(xi_j) = w_j D[j, i] (eq. lobatto-advection, transposed)."""
    return (D * w[:, None]).T


def operators(n):
    """All reference-element operators for n LGL nodes, as a dict."""
    xi, w = lgl_nodes_weights(n)
    D = derivative_matrix(xi)
    Minv = mass_inverse(xi, w)
    S = stiffness(w, D)
    ups = Minv @ S
    xi_cols = Minv[:, [0, n - 1]]
    return {"n": n, "xi": xi, "w": w, "D": D, "Minv": Minv, "S": S,
            "A": S.T.copy(), "Ups": ups, "Xi": xi_cols}
