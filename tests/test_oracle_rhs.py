"""Pins of oracle.rhs: dense brute-force assembly, conservation, exact solutions."""
import math

import numpy as np
import pytest

from oracle import brute, cfl, grid, lgl, rhs, rk


@pytest.mark.parametrize("n,ne,vbc", [(2, (3, 3), "periodic"), (3, (3, 4), "periodic"),
                                      (4, (2, 3), "zero_inflow"), (3, (3, 3), "zero_inflow"),
                                      (10, (2, 2), "periodic"), (12, (2, 2), "zero_inflow")])
def test_rhs_matches_brute_force_1d1v(n, ne, vbc):
    rng = np.random.default_rng(10 * n + ne[0])
    g = grid.PhaseGrid(1, n, list(ne), [0.0, -2.0], [2 * math.pi, 2.5], vbc=vbc)
    f = rng.random(g.shape)
    E = rng.standard_normal((ne[0], n))
    r1 = rhs.rhs(g, lgl.operators(n), f, E)
    r2 = brute.brute_rhs(g, f, E)
    assert np.max(np.abs(r1 - r2)) <= 1e-12 * np.max(np.abs(r2))


@pytest.mark.parametrize("n,ne,B,vbc", [(2, (2, 3, 3), 0.7, "periodic"), (3, (2, 3, 2), -1.3, "periodic"),
                                        (3, (2, 2, 3), 0.4, "zero_inflow")])
def test_rhs_matches_brute_force_1d2v(n, ne, B, vbc):
    rng = np.random.default_rng(100 * n + ne[1])
    g = grid.PhaseGrid(2, n, list(ne), [0.0, -2.0, -1.5], [2 * math.pi, 2.0, 2.5], omega_c=B, vbc=vbc)
    f = rng.random(g.shape)
    E = rng.standard_normal((ne[0], n))
    r1 = rhs.rhs(g, lgl.operators(n), f, E)
    r2 = brute.brute_rhs(g, f, E)
    assert np.max(np.abs(r1 - r2)) <= 1e-12 * np.max(np.abs(r2))


@pytest.mark.parametrize("nv,n", [(1, 4), (1, 7), (2, 3), (2, 5)])
def test_discrete_mass_conservation(nv, n):
    rng = np.random.default_rng(nv * 31 + n)
    if nv == 1:
        g = grid.PhaseGrid(1, n, [5, 6], [0.0, -4.0], [3.0, 4.0])
    else:
        g = grid.PhaseGrid(2, n, [3, 4, 5], [0.0, -4.0, -4.0], [3.0, 4.0, 4.0], omega_c=0.9)
    f = rng.random(g.shape)
    E = rng.standard_normal((g.axes[0].N, n))
    r = rhs.rhs(g, lgl.operators(n), f, E)
    W = g.weights()
    assert abs(np.sum(W * r)) <= 1e-13 * np.sum(W * np.abs(r))


def _free_stream_error(n, nx, t_end=1.0, dt=None):
    L = 2 * math.pi
    g = grid.PhaseGrid(1, n, [nx, 4], [0.0, -1.0], [L, 1.0])
    x, v = g.coords()
    f0 = lambda xx, vv: (1.0 + 0.5 * np.sin(xx)) * np.exp(-vv * vv)
    f = f0(x, v) + 0 * v
    ops = lgl.operators(n)
    dt = dt or 0.2 * g.axes[0].dx
    steps = int(round(t_end / dt))
    dt = t_end / steps
    Ez = np.zeros((nx, n))
    for _ in range(steps):
        f = rk.ssprk3_step(g, ops, f, dt, E_override=Ez)
    exact = f0(x - v * t_end, v) + 0 * v
    return np.sqrt(np.sum(g.weights() * (f - exact) ** 2))


def test_free_streaming_converges():
    # E = 0, B = 0: f(x, v, t) = f0(x - v t, v); error falls at high order in h
    e1 = _free_stream_error(3, 8, dt=0.01)
    e2 = _free_stream_error(3, 16, dt=0.005)
    assert e1 < 1e-2
    assert math.log2(e1 / e2) > 2.5      # third-order (n = 3) spatial convergence
    assert _free_stream_error(6, 8, dt=0.002) < 1e-6


def _gyration_error(n, nv_el, t_end):
    # x-uniform, E = 0, B = omega: rigid counter-clockwise rotation in (u, v)
    B = 1.0
    g = grid.PhaseGrid(2, n, [1, nv_el, nv_el], [0.0, -6.0, -6.0], [1.0, 6.0, 6.0], omega_c=B)
    _, u, v = g.coords()
    f0 = lambda uu, vv: np.exp(-((uu - 1.5) ** 2 + (vv + 0.5) ** 2) / 1.0)
    f = f0(u, v) + 0 * (u + v)
    f = np.broadcast_to(f, g.shape).copy()
    ops = lgl.operators(n)
    dt = 0.5 * cfl.dt_max(g, 0.0)
    steps = int(math.ceil(t_end / dt))
    dt = t_end / steps
    Ez = np.zeros((1, n))
    for _ in range(steps):
        f = rk.ssprk3_step(g, ops, f, dt, E_override=Ez)
    c, s = math.cos(B * t_end), math.sin(B * t_end)
    exact = f0(u * c + v * s, -u * s + v * c) + 0 * f
    return np.sqrt(np.sum(g.weights() * (f - exact) ** 2)) / np.sqrt(np.sum(g.weights() * exact ** 2))


def test_gyration_is_rotation():
    e_coarse = _gyration_error(4, 8, math.pi / 2)
    e_fine = _gyration_error(4, 16, math.pi / 2)
    assert e_fine < 5e-3
    assert e_coarse / e_fine > 6.0          # ~ h^4 convergence of the rotation
