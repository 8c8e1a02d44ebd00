"""Moments and energies of a DG phase-space state by LGL quadrature, FP64.

Test infrastructure (see ``oracle/__init__``).

The paper plots the domain-integrated electric field energy (Sec. 6, energy
figure) without defining it; the reading used here is W_E = 1/2 int E^2 dx by
nodal LGL quadrature.  Mass is int int f, kinetic energy 1/2 int |v|^2 f and the
L2 norm int f^2, all by the product LGL rule (exact for the interpolant's
polynomial integrands up to degree 2n-3 per axis).

Pinned by tests/test_oracle_diag.py: the ring-distribution moments of App. B
(closed forms with Gamma functions), Gaussian moments, and the field energy of
a linear field (exactly L^3/6: pins the factor 1/2 and the weights w dx/2) and
of a single Fourier mode (A^2 L/4).
"""
import numpy as np

from . import rhs as rhs_mod


def mass(grid, f):
    return float(np.sum(grid.weights() * f))


def field_energy(grid, E):
    ax = grid.axes[0]
    return 0.5 * float(np.sum(ax.qw * np.asarray(E).reshape(ax.N, ax.n) ** 2))


def kinetic_energy(grid, f):
    c = grid.coords()
    v2 = sum(ci ** 2 for ci in c[1:])
    return 0.5 * float(np.sum(grid.weights() * v2 * f))


def l2sq(grid, f):
    return float(np.sum(grid.weights() * f * f))


def all_diagnostics(grid, f, E):
    return {"mass": mass(grid, f), "field_energy": field_energy(grid, E),
            "kinetic_energy": kinetic_energy(grid, f), "l2sq": l2sq(grid, f),
            "max_abs_E": float(np.max(np.abs(E)))}
