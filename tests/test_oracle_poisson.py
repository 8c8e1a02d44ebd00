"""Pins of oracle.poisson: exact Fourier coefficients, closed form, convergence."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import grid, lgl, poisson
from tests.golden import paper_value


@pytest.mark.parametrize("n,N", [(2, 7), (3, 10), (5, 6), (8, 12)])
def test_sawtooth_coefficients_exact(n, N):
    # f(x) = x on [0, L) is a polynomial on every element -> interpolated exactly;
    # its Fourier coefficients are c_p = i / k_p (p != 0), c_0 = L / 2.
    L = 3.0
    ax = grid.Axis(0.0, L, N, n)
    c, ps, k = poisson.fourier_coefficients(ax, ax.nodes, N)
    for ci, p, kp in zip(c, ps, k):
        expect = L / 2 if p == 0 else 1j / kp
        assert abs(ci - expect) < 1e-13, (p, ci, expect)
    if n >= 3:
        # f = x^2: c_p = i L / k_p + 2 / k_p^2
        c2, _, _ = poisson.fourier_coefficients(ax, ax.nodes ** 2, N)
        for ci, p, kp in zip(c2, ps, k):
            expect = L * L / 3 if p == 0 else 1j * L / kp + 2 / kp ** 2
            assert abs(ci - expect) < 1e-12, (p, ci, expect)


@pytest.mark.parametrize("n,N", [(2, 5), (4, 8), (8, 10), (9, 16)])
def test_connection_tensor_closed_form(n, N):
    """Quadrature T equals eq. spectral_transform (spherical Bessel closed form)."""
    L = 2.5
    ax = grid.Axis(0.0, L, N, n)
    T, ps, k = poisson.connection_tensor(ax, N)
    x, w = ax.xi, ax.w
    gamma = np.array([2.0 / (2 * s + 1) for s in range(n - 1)] + [2.0 / (n - 1)])
    for ip, (p, kp) in enumerate(zip(ps, k)):
        for m in range(N):
            kap = kp / ax.J
            ssum = sum((-1j) ** s * lgl.legendre(s, x) * sp.spherical_jn(s, abs(kap)) * (np.sign(kap) ** s if kap != 0 else 1)
                       / gamma[s] for s in range(n))
            closed = (ax.dx / L) * np.exp(-1j * kp * ax.mid[m]) * w * ssum
            assert np.max(np.abs(T[ip, m] - closed)) < 1e-14


def test_T_annihilates_constants():
    ax = grid.Axis(-1.0, 2.0, 9, 6)
    c, ps, _ = poisson.fourier_coefficients(ax, np.ones((9, 6)), 9)
    for ci, p in zip(c, ps):
        assert abs(ci - (1.0 if p == 0 else 0.0)) < 1e-15


def _poisson_errors(n, N):
    ax = grid.Axis(0.0, 1.0, N, n)
    src = np.sin(2 * math.pi * ax.nodes)
    Phi, E, _ = poisson.solve(ax, src, pmax=N)
    # broken L2 norm (eq. broken_l2): mean over elements of per-element L2 norms,
    # integrated with a fine Gauss rule on the interpolants
    eta, om = np.polynomial.legendre.leggauss(30)
    ell = np.stack([lgl.lagrange_eval(ax.xi, j, eta) for j in range(n)], axis=1)
    errs = []
    for vals, exact in ((Phi, lambda x: -np.sin(2 * math.pi * x) / (4 * math.pi ** 2)),
                        (E, lambda x: np.cos(2 * math.pi * x) / (2 * math.pi))):
        tot = 0.0
        for m in range(N):
            xq = ax.mid[m] + eta / ax.J
            d = ell @ vals[m] - exact(xq)
            tot += math.sqrt(np.sum(om * d * d) / ax.J)
        errs.append(tot / N)
    return errs


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_poisson_sine_hp_convergence(n):
    """Phi'' = sin(2 pi x): error falls like dx^(n+1/2) (Sec. 5.3.2, Poisson figure)."""
    Ns = [10, 15, 20, 25]
    e = np.array([_poisson_errors(n, N) for N in Ns])
    order = n + paper_value("poisson_convergence_order_offset")["value"]   # n + 1/2
    for col in range(2):
        slope = -np.polyfit(np.log(Ns), np.log(e[:, col]), 1)[0]
        assert order - 0.2 < slope < order + 0.25, (n, col, slope, e[:, col])
    assert e[-1, 1] < 1e-4


def test_field_is_continuous_for_noisy_source():
    # the Fourier series is single valued, so E is C^0 across element faces
    rng = np.random.default_rng(3)
    ax = grid.Axis(-math.pi, math.pi, 10, 8)
    src = np.sin(ax.nodes) + rng.standard_normal(ax.nodes.shape)
    _, E, _ = poisson.solve(ax, src - src.mean())
    assert np.max(np.abs(E[:-1, -1] - E[1:, 0])) < 1e-12
