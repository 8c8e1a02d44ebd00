"""Pins of oracle.rk: third-order time accuracy and the Landau damping rate."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import diagnostics, grid, lgl, rhs, rk


def test_ssprk3_is_third_order():
    # same semi-discrete system at dt, dt/2 against a dt/16 reference
    n = 4
    g = grid.PhaseGrid(1, n, [6, 2], [0.0, -1.0], [2 * math.pi, 1.0])
    x, v = g.coords()
    f0 = (1.0 + 0.5 * np.sin(x)) * np.exp(-v * v) + 0 * v
    ops = lgl.operators(n)
    Ez = np.zeros((6, n))

    def run(dt, T=0.5):
        f = f0.copy()
        for _ in range(int(round(T / dt))):
            f = rk.ssprk3_step(g, ops, f, dt, E_override=Ez)
        return f
    ref = run(0.05 / 16)
    e1 = np.max(np.abs(run(0.05) - ref))
    e2 = np.max(np.abs(run(0.025) - ref))
    assert 2.8 < math.log2(e1 / e2) < 3.3


def landau_root(k):
    """Least-damped root of 1 + (1 + zeta Z(zeta)) / k^2 = 0, zeta = omega / (k sqrt 2)."""
    Z = lambda z: 1j * math.sqrt(math.pi) * sp.wofz(z)
    eps = lambda w: 1.0 + (1.0 + (w / (k * math.sqrt(2))) * Z(w / (k * math.sqrt(2)))) / (k * k)
    w0, w1 = 1.4 - 0.15j, 1.41 - 0.16j
    for _ in range(60):
        f0, f1 = eps(w0), eps(w1)
        w0, w1 = w1, w1 - f1 * (w1 - w0) / (f1 - f0)
        if abs(w1 - w0) < 1e-14:
            break
    return w1


@pytest.mark.slow
def test_linear_landau_damping_rate():
    """1D1V, k = 0.5, n = 4, 16 x 32 elements: field energy decays at 2 gamma."""
    wroot = landau_root(0.5)
    assert abs(wroot.real - 1.4157) < 1e-3 and abs(wroot.imag + 0.1534) < 1e-3
    n = 4
    g = grid.PhaseGrid(1, n, [16, 32], [0.0, -8.0], [4 * math.pi, 8.0])
    x, v = g.coords()
    f = (1.0 + 0.01 * np.cos(0.5 * x)) * np.exp(-0.5 * v * v) / math.sqrt(2 * math.pi)
    ops = lgl.operators(n)
    dt, steps = 0.01, 2000
    t = [0.0]
    W = [diagnostics.field_energy(g, rk.field(g, f))]
    m0 = diagnostics.mass(g, f)
    for s in range(steps):
        f = rk.ssprk3_step(g, ops, f, dt)
        t.append((s + 1) * dt)
        W.append(diagnostics.field_energy(g, rk.field(g, f)))
    assert abs(diagnostics.mass(g, f) - m0) < 1e-12 * m0
    t, W = np.array(t), np.array(W)
    pk = [i for i in range(1, len(W) - 1) if W[i] > W[i - 1] and W[i] >= W[i + 1] and 1.0 < t[i] < 19.0]
    slope = np.polyfit(t[pk], np.log(W[pk]), 1)[0]
    assert abs(slope / (2 * wroot.imag) - 1.0) < 0.03, (slope, 2 * wroot.imag)
    # oscillation frequency: field-energy peaks are half a period apart
    period = 2 * np.mean(np.diff(t[pk]))
    assert abs(2 * math.pi / period / wroot.real - 1.0) < 0.02
