"""Pins of oracle.diagnostics: App. B ring moments and Gaussian moments."""
import math

import numpy as np
import pytest

from oracle import diagnostics, grid
from tests.golden import paper_value


def _vgrid(n=8, ne=40, vmax=12.0):
    return grid.PhaseGrid(2, n, [1, ne, ne], [0.0, -vmax, -vmax], [1.0, vmax, vmax])


@pytest.mark.parametrize("j,alpha", [(6, 1.0), (3, 0.8)])
def test_ring_moments_appendix_b(j, alpha):
    g = _vgrid()
    _, u, v = g.coords()
    vp = np.sqrt(u * u + v * v)
    f0 = (vp ** 2 / (2 * alpha ** 2)) ** j * np.exp(-vp ** 2 / (2 * alpha ** 2)) / (2 * math.pi * alpha ** 2 * math.factorial(j))
    f0 = np.broadcast_to(f0, g.shape)
    W = g.weights()
    assert abs(np.sum(W * f0) - 1.0) < 1e-10
    ratio = math.gamma(j + 1.5) / math.gamma(j + 1)
    mean_v = np.sum(W * vp * f0)
    assert abs(mean_v - math.sqrt(2) * alpha * ratio) < 1e-8
    centred = 0.5 * np.sum(W * (vp - mean_v) ** 2 * f0)
    assert abs(centred - alpha ** 2 * (j + 1 - ratio ** 2)) < 1e-8
    # leading-order estimate quoted in App. B: alpha^2/4 per unit length
    # (0.25 at alpha = 1, the thermal energy in the energy figure's caption)
    th = paper_value("ring_thermal_energy_per_length")
    est = th["value"] * (alpha / th["alpha"]) ** 2
    assert abs(centred / est - 1) < 1.0 / (8 * j) + 0.02


def test_maxwellian_mass_and_energy():
    g = _vgrid(6, 24, 9.0)
    _, u, v = g.coords()
    f = np.broadcast_to(np.exp(-(u * u + v * v) / 2) / (2 * math.pi), g.shape)
    assert abs(diagnostics.mass(g, f) - 1.0) < 1e-12
    assert abs(diagnostics.kinetic_energy(g, f) - 1.0) < 1e-11
    assert abs(diagnostics.l2sq(g, f) - 1.0 / (4 * math.pi)) < 1e-12


@pytest.mark.parametrize("n,N,L", [(4, 5, 3.7), (3, 7, 11.0), (6, 2, 0.9)])
def test_field_energy_closed_form_linear_field(n, N, L):
    # E(x) = x - x0 on [x0, x0 + L): a polynomial of degree 1 in every element,
    # so its nodal interpolant is exact and E^2 (degree 2 <= 2n - 3 for n >= 3)
    # is integrated exactly by the LGL rule: W_E = 1/2 int_0^L s^2 ds = L^3 / 6.
    # The element width L/N differs from 2, so weights w_j instead of
    # w_j dx/2 fail, and so does a dropped factor 1/2.
    x0 = -1.3
    g = grid.PhaseGrid(1, n, [N, 4], [x0, -1.0], [x0 + L, 1.0])
    E = g.axes[0].nodes - x0
    assert abs(diagnostics.field_energy(g, E) - L ** 3 / 6.0) < 1e-12 * L ** 3


def test_field_energy_single_mode_parseval():
    # E = A sin(k x + phi) on one period: W_E = A^2 L / 4 (spectral accuracy
    # of the LGL rule on a smooth periodic integrand).
    L, A, phi = 4 * math.pi, 0.37, 0.4
    g = grid.PhaseGrid(1, 8, [12, 4], [0.0, -1.0], [L, 1.0])
    x = g.axes[0].nodes
    E = A * np.sin(2 * math.pi / L * 3 * x + phi)
    assert abs(diagnostics.field_energy(g, E) - A * A * L / 4) < 1e-12
