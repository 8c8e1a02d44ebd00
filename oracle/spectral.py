"""Spectral tools on the x grid built on the connection tensor, FP64.

Test infrastructure (see ``oracle/__init__``).

Sec. 5.3 names, besides the Poisson solve, a global filter for anti-aliasing
as an application of the transform c_p = T_p^{mj} f_mj (eq. spectral_transform;
T here by brute-force Gauss-Legendre quadrature, ``oracle.poisson``).  The
filter replaces a nodal x profile by its Fourier series truncated at pmax
(eq. fourier_series) with mode weights sigma_|p|, evaluated at the nodes:

    f_out(x_mj) = sum_{|p| <= pmax} sigma_|p| c_p e^{i k_p x_mj},  sigma_0 = 1.

Pinned by tests/test_oracle_spectral.py: a trigonometric polynomial passes
the all-ones filter to the accuracy of its nodal interpolation (which
converges at the rate of the basis), a zero weight removes exactly its mode,
and the transform reproduces the closed-form Fourier coefficients of the
elliptic cosine up to the aliasing limit of the errors figure.
"""
import numpy as np

from . import poisson


def filter_x(axis, f, sigma):
    """Apply the x filter to an array whose two leading axes are (element, node) of x."""
    sigma = np.asarray(sigma, dtype=np.float64)
    pmax = sigma.size
    f = np.asarray(f, dtype=np.float64)
    rest = f.shape[2:]
    cols = f.reshape(axis.N * axis.n, -1)
    T, ps, k = poisson.connection_tensor(axis, pmax)
    Tm = T.reshape(len(ps), axis.N * axis.n)                 # (P, nodes)
    c = Tm @ cols                                            # (P, columns)
    w = np.concatenate([sigma[::-1], [1.0], sigma])          # sigma_|p| for p = -pmax..pmax
    x = axis.nodes.reshape(-1)
    S = np.exp(1j * np.outer(x, k))                          # (nodes, P)
    out = (S @ (w[:, None] * c)).real
    return out.reshape(f.shape[:2] + rest)
