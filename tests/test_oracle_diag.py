"""Pins of oracle.diagnostics: App. B ring moments and Gaussian moments."""
import math

import numpy as np
import pytest

from oracle import diagnostics, grid


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
    # leading-order estimates quoted in App. B
    assert abs(centred / (alpha ** 2 / 4) - 1) < 1.0 / (8 * j) + 0.02


def test_maxwellian_mass_and_energy():
    g = _vgrid(6, 24, 9.0)
    _, u, v = g.coords()
    f = np.broadcast_to(np.exp(-(u * u + v * v) / 2) / (2 * math.pi), g.shape)
    assert abs(diagnostics.mass(g, f) - 1.0) < 1e-12
    assert abs(diagnostics.kinetic_energy(g, f) - 1.0) < 1e-11
    assert abs(diagnostics.l2sq(g, f) - 1.0 / (4 * math.pi)) < 1e-12
