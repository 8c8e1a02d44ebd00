"""Stability limit of SSP-RK3 with upwind weak-form LGL DG, FP64.

Test infrastructure (see ``oracle/__init__``).

Sec. 6 takes order-dependent CFL numbers from the literature without printing
them.  This module recomputes the limit from its definition: for u_t + u_x = 0
on a periodic grid of identical elements, a Fourier (Bloch) mode
u_{m+1} = e^{i theta} u_m turns the weak-form operator of one element into
    L(theta) = J [ Upsilon + e^{-i theta} Xi_0 e_{n-1}^T - Xi_1 e_{n-1}^T ]
(upwind: the left face takes the left neighbour's last node, the right face
the element's own last node).  RK3 is stable when every dt * lambda lies in
{z : |1 + z + z^2/2 + z^3/6| <= 1}.  With J = 2/dx the limit has the form
dt_max = C_n dx / |a|; C_n is found by bisection over a theta sweep.

Pinned by tests/test_oracle_cfl.py: time-stepping the oracle's own RHS just
below and just above the limit (bounded vs growing), and the P1/RK3 value.
"""
import numpy as np

from . import lgl


def bloch_eigenvalues(n, nthetas=721):
    ops = lgl.operators(n)
    ups, xi = ops["Ups"], ops["Xi"]
    e_last = np.zeros(n)
    e_last[-1] = 1.0
    lams = []
    for th in np.linspace(0.0, 2.0 * np.pi, nthetas):
        Lm = ups + np.exp(-1j * th) * np.outer(xi[:, 0], e_last) - np.outer(xi[:, 1], e_last)
        lams.append(np.linalg.eigvals(Lm))     # J = 1
    return np.concatenate(lams)


def rk3_amplification(z):
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0


def courant_number(n):
    """C_n such that dt <= C_n dx / |a| is RK3-stable (J = 2/dx)."""
    lam = bloch_eigenvalues(n)
    lo, hi = 0.0, 2.0
    for _ in range(60):
        c = 0.5 * (lo + hi)
        z = 2.0 * c * lam                    # dt * lambda with J = 2/dx, dt = c dx
        if np.max(np.abs(rk3_amplification(z))) <= 1.0 + 1e-12:
            lo = c
        else:
            hi = c
    return lo


def dt_max(grid, max_abs_E):
    """Largest stable dt for the phase-space speeds bounded as in eq. vlasov."""
    cn = courant_number(grid.n)
    axes = grid.axes
    vmax = [max(abs(a.lo), abs(a.hi)) for a in axes[1:]]
    if grid.nv == 1:
        rate = vmax[0] / axes[0].dx + max_abs_E / axes[1].dx
    else:
        B = abs(grid.omega_c)
        rate = (vmax[0] / axes[0].dx + (max_abs_E + vmax[1] * B) / axes[1].dx
                + vmax[0] * B / axes[2].dx)
    return cn / rate
