"""Shu-Osher SSP-RK3 time stepping of the Vlasov-Poisson system, FP64.

Test infrastructure (see ``oracle/__init__``).

Sec. 6: the weak-form semi-discrete equation is advanced with the three-stage
strong-stability-preserving Runge-Kutta method of Shu and Osher, and Poisson's
equation is solved at every stage from that stage's argument.  The paper cites
the scheme without writing its coefficients; the standard Shu-Osher form is
    u1      = u + dt L(u)
    u2      = 3/4 u + 1/4 (u1 + dt L(u1))
    u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2)).

Pinned by tests/test_oracle_rk.py: third-order convergence in dt on free
streaming, and through the Landau damping rate.
"""
import numpy as np

from . import rhs as rhs_mod
from . import poisson


def field(grid, f, pmax=None, E_override=None):
    if E_override is not None:
        return np.asarray(E_override, dtype=np.float64).reshape(grid.axes[0].N, grid.n)
    nd = rhs_mod.density(grid, f)
    E, _ = poisson.field_from_density(grid, nd, pmax)
    return E


def L(grid, ops, f, pmax=None, E_override=None):
    return rhs_mod.rhs(grid, ops, f, field(grid, f, pmax, E_override))


def ssprk3_step(grid, ops, f, dt, pmax=None, E_override=None):
    f = np.asarray(f, dtype=np.float64)
    u1 = f + dt * L(grid, ops, f, pmax, E_override)
    u2 = 0.75 * f + 0.25 * (u1 + dt * L(grid, ops, u1, pmax, E_override))
    return f / 3.0 + (2.0 / 3.0) * (u2 + dt * L(grid, ops, u2, pmax, E_override))
