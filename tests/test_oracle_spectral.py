"""Pins of the connection-tensor tools (Sec. 5.3.1 and its errors figure).

* Elliptic cosine cn(4 K x | m) on [-1/2, 1/2], sqrt(m) = 1 - 1e-6, N = 20
  elements: its Fourier coefficients in closed form (DLMF 22.11.2:
  cn(z|m) = (pi / (K sqrt m)) sum_n sech((2n + 1) pi K' / (2K)) cos((2n + 1) pi z / (2K)),
  so c_{+-(2n+1)} = (pi / (2 K sqrt m)) sech((2n + 1) pi K' / (2K)) and the even
  coefficients vanish).  The paper prints the sech argument without the
  factor 1/2 (read as a typo: the standard expansion is used).  Checked, as
  the figure states: even modes at the rounding level (1e-16 of the largest
  coefficient); the first local minimum of the odd-mode error (the aliasing
  point) beyond the DFT Nyquist mode p = N/2 = 10 for every n, and beyond
  2 x 10 = N for n >= 6 (``p_max ~ N``).
* The x filter of oracle.spectral: all-ones weights pass a trigonometric
  polynomial up to its interpolation error, a zero weight removes its mode.
"""
import math

import numpy as np
import pytest
from scipy import special

from oracle import grid, poisson, spectral
from paper_2202_13532_amd import inputs

SQRT_M = 1.0 - 1e-6
N_ELEM = 20


def cn_coefficients(pmax, sqrt_m=SQRT_M):
    m = sqrt_m * sqrt_m
    K, Kp = special.ellipk(m), special.ellipk(1.0 - m)
    c = np.zeros(pmax + 1)
    for p in range(1, pmax + 1, 2):
        c[p] = 0.5 * math.pi / (K * sqrt_m) / math.cosh(0.5 * math.pi * p * Kp / K)
    return c


def aliasing_point(err_odd, odd):
    for i in range(1, len(odd) - 1):
        if err_odd[i] < err_odd[i - 1] and err_odd[i] <= err_odd[i + 1]:
            return int(odd[i])
    return None


def cn_study(n, pmax=60):
    ax = grid.Axis(-0.5, 0.5, N_ELEM, n)
    vals = inputs.elliptic_cosine(ax.nodes, SQRT_M)
    c, ps, _ = poisson.fourier_coefficients(ax, vals, pmax)
    cp = c[pmax + 1:]
    ce = cn_coefficients(pmax)[1:]
    odd = np.arange(1, pmax + 1, 2)
    err = np.abs(cp[odd - 1] - ce[odd - 1]) / np.abs(ce[odd - 1])
    even = np.max(np.abs(cp[1::2])) / np.max(np.abs(ce))
    return err, odd, even, cp


def test_cn_closed_form_coefficients_match_quadrature():
    # the closed form itself, against direct quadrature of cn on a fine grid
    x = (np.arange(200000) + 0.5) / 200000 - 0.5
    f = inputs.elliptic_cosine(x, SQRT_M)
    ce = cn_coefficients(9)
    for p in range(1, 10):
        cq = np.mean(f * np.exp(-2j * math.pi * p * x))
        assert abs(cq - ce[p]) < 1e-9, p


@pytest.mark.parametrize("n", range(2, 10))
def test_aliasing_study_of_the_errors_figure(n):
    err, odd, even, _ = cn_study(n)
    assert even < 1e-14
    ap = aliasing_point(err, odd)
    assert ap is not None and ap > N_ELEM // 2
    if n >= 6:
        assert ap > N_ELEM
        assert err[0] < 1e-7          # mode 1 essentially exact at high order


@pytest.mark.parametrize("n,N", [(4, 12), (7, 9), (9, 6)])
def test_x_filter_pass_and_stop(n, N):
    ax = grid.Axis(0.0, 3.0, N, n)
    k = 2 * math.pi / 3.0
    x = ax.nodes
    f = 1.0 + 0.5 * np.cos(k * x) + 0.25 * np.sin(3 * k * x + 0.3)
    pmax = N
    out = spectral.filter_x(ax, f, np.ones(pmax))
    # the DG interpolant differs from the trigonometric polynomial by its
    # interpolation error; the filter returns the polynomial's nodal values
    assert np.max(np.abs(out - f)) < 10.0 * (3.0 * k * ax.dx) ** n / math.factorial(n)
    sig = np.ones(pmax)
    sig[2] = 0.0                     # remove p = 3
    out3 = spectral.filter_x(ax, f, sig)
    ref = 1.0 + 0.5 * np.cos(k * x)
    assert np.max(np.abs(out3 - ref)) < 10.0 * (3.0 * k * ax.dx) ** n / math.factorial(n)
    # zero weights leave the mean
    out0 = spectral.filter_x(ax, f, np.zeros(pmax))
    c0 = np.sum(f * ax.qw) / 3.0
    assert np.max(np.abs(out0 - c0)) < 1e-14
