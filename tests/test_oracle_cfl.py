"""Pins of oracle.cfl: the computed limit separates bounded from growing runs."""
import math

import numpy as np
import pytest

from oracle import cfl, grid, lgl, rk


@pytest.mark.parametrize("n", [2, 4, 8])
def test_limit_separates_stable_and_unstable(n):
    # free streaming in x with speeds = v nodes in [-1, 1] (max |v| = 1)
    g = grid.PhaseGrid(1, n, [8, 1], [0.0, -1.0], [1.0, 1.0])
    ops = lgl.operators(n)
    dtm = cfl.dt_max(g, 0.0)
    assert abs(dtm - cfl.courant_number(n) * g.axes[0].dx) < 1e-15
    Ez = np.zeros((8, n))
    rng = np.random.default_rng(n)
    f0 = rng.standard_normal(g.shape)

    def growth(frac, steps):
        f = f0.copy()
        for _ in range(steps):
            f = rk.ssprk3_step(g, ops, f, frac * dtm, E_override=Ez)
        return np.linalg.norm(f) / np.linalg.norm(f0)
    assert growth(0.98, 1500) <= 1.0 + 1e-9
    assert growth(1.10, 1500) > 10.0


def test_known_p1_value_and_monotone_in_n():
    cs = [cfl.courant_number(n) for n in range(2, 10)]
    # linear (P1) upwind DG with SSP-RK3: about 0.409 (Cockburn-Shu stability table)
    assert abs(cs[0] - 0.409) < 1e-3
    assert all(a > b for a, b in zip(cs, cs[1:]))
    # 1/(2n-1) would be unstable for n >= 4
    assert all(cfl.courant_number(n) < 1.0 / (2 * n - 1) for n in range(4, 10))
