"""LGL -> Fourier connection tensor and the spectral Poisson solve, FP64.

Test infrastructure (see ``oracle/__init__``).

Sec. 5.3: the piecewise interpolant f(x) = (+)_m sum_j f_mj l_j(x) has the
Fourier coefficients c_p = (1/L) int_0^L f(x) e^{-i k_p x} dx, k_p = 2 pi p / L
(eq. fourier_series), i.e. c_p = T_p^{mj} f_mj with
    T_p^{mj} = (1/L) int_{element m} l_j(xi(x)) e^{-i k_p x} dx.
The paper evaluates this integral in closed form with spherical Bessel
functions (eq. spectral_transform).  The oracle deliberately does NOT use that
formula: it integrates l_j e^{-ikx} by brute-force Gauss-Legendre quadrature
with many more points than needed, so it is an independent check of the
closed form used by the library.

Poisson (eq. poisson, eq. fourier_poisson): d_xx Phi = n - 1 with
-k_p^2 Phi_p = c_p, summed for 0 < |p| <= p_max (the p = 0 mode is the neutral
mean and is excluded):
    Phi_mj = sum_p -k_p^-2 c_p e^{i k_p x_mj}               (eq. poisson_solution)
    E_mj   = sum_p -(i k_p)^-1 c_p e^{i k_p x_mj}           (eq. electric_sol)

Pinned by tests/test_oracle_poisson.py: exact Fourier coefficients of periodic
polynomial sawtooth data, the closed form with scipy's spherical Bessel
functions, T 1 = 0 for p != 0, the Phi'' = sin(2 pi x) benchmark and its
h-convergence, and C^0 continuity of E.
"""
import numpy as np

from . import lgl


_T_CACHE = {}


def connection_tensor(axis, pmax, extra_points=24):
    """T[p_index, m, j] for p = -pmax..pmax (p_index = p + pmax), complex128."""
    key = (axis.lo, axis.hi, axis.N, axis.n, int(pmax), extra_points)
    if key not in _T_CACHE:
        _T_CACHE[key] = _connection_tensor(axis, pmax, extra_points)
    return _T_CACHE[key]


def _connection_tensor(axis, pmax, extra_points):
    N, n, L = axis.N, axis.n, axis.L
    q = max(n + extra_points, 32)
    eta, omega = np.polynomial.legendre.leggauss(q)
    ell = np.stack([lgl.lagrange_eval(axis.xi, j, eta) for j in range(n)])   # (n, q)
    ps = np.arange(-pmax, pmax + 1)
    k = 2.0 * np.pi * ps / L
    T = np.zeros((len(ps), N, n), dtype=np.complex128)
    for m in range(N):
        xq = axis.mid[m] + eta / axis.J                                         # (q,)
        phase = np.exp(-1j * k[:, None] * xq[None, :])                          # (P, q)
        # (dx/2) sum_q omega_q l_j(eta_q) e^{-ik x_q} / L
        T[:, m, :] = (phase * omega[None, :]) @ ell.T / axis.J / L
    return T, ps, k


def fourier_coefficients(axis, values, pmax):
    T, ps, k = connection_tensor(axis, pmax)
    c = np.tensordot(T, np.asarray(values, dtype=np.float64).reshape(axis.N, axis.n),
                     axes=([1, 2], [0, 1]))
    return c, ps, k


def solve(axis, source, pmax=None):
    """Spectral solution of Phi'' = source; returns (Phi, E, c) at the nodes."""
    pmax = axis.N if pmax is None else int(pmax)
    c, ps, k = fourier_coefficients(axis, source, pmax)
    x = axis.nodes
    Phi = np.zeros(x.shape, dtype=np.complex128)
    E = np.zeros(x.shape, dtype=np.complex128)
    for i, p in enumerate(ps):
        if p == 0:
            continue
        mode = np.exp(1j * k[i] * x)
        Phi += -c[i] / k[i] ** 2 * mode
        E += -(c[i] / (1j * k[i])) * mode
    return Phi.real, E.real, c


def field_from_density(grid, ndens, pmax=None):
    """E at the x nodes from the electron density n_mj (source n - 1)."""
    _, E, c = solve(grid.axes[0], np.asarray(ndens) - 1.0, pmax)
    return E, c
