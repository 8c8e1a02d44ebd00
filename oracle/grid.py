"""Element geometry of a rectilinear LGL grid, FP64.

Test infrastructure (see ``oracle/__init__``).

Sec. 2 (isoparametric map with Jacobian J = 2 / dx) and Sec. 5.3 (affine map
xi = J_m (x - xbar_m), xbar_m the element midpoint): element m of an axis on
[lo, hi] with N equal elements spans [lo + m dx, lo + (m + 1) dx], its node j
sits at x_mj = lo + (m + 1/2) dx + xi_j / J.

Pinned indirectly: every physics test (free streaming, gyration, Poisson
convergence, Landau damping) fails if the coordinates are wrong.
"""
import numpy as np

from . import lgl


class Axis:
    def __init__(self, lo, hi, nelem, n):
        self.lo, self.hi, self.N, self.n = float(lo), float(hi), int(nelem), int(n)
        self.L = self.hi - self.lo
        self.dx = self.L / self.N
        self.J = 2.0 / self.dx
        self.xi, self.w = lgl.lgl_nodes_weights(self.n)
        mid = self.lo + (np.arange(self.N) + 0.5) * self.dx
        self.nodes = mid[:, None] + self.xi[None, :] / self.J      # (N, n)
        self.mid = mid
        self.qw = np.broadcast_to(self.w / self.J, (self.N, self.n)).copy()  # quadrature weights

    def flat_nodes(self):
        return self.nodes.reshape(-1)


class PhaseGrid:
    """1D1V (nv=1: axes x, v) or 1D2V (nv=2: axes x, u, v) phase space.

    The state is stored as [N_x, n, N_u, n, N_v, n] (1D2V) or [N_x, n, N_v, n]
    (1D1V): element index then node index per axis, row-major (Sec. 3.1).
    """

    def __init__(self, nv, n, nelem, lo, hi, omega_c=0.0, vbc="periodic"):
        self.nv = int(nv)
        self.n = int(n)
        naxes = 1 + self.nv
        self.axes = [Axis(lo[a], hi[a], nelem[a], n) for a in range(naxes)]
        self.omega_c = float(omega_c)
        self.vbc = vbc
        self.shape = tuple(s for a in self.axes for s in (a.N, a.n))

    @property
    def x(self):
        return self.axes[0]

    def dof(self):
        return int(np.prod(self.shape))

    def coords(self):
        """Broadcastable node-coordinate arrays, one per axis, in state layout."""
        out = []
        naxes = len(self.axes)
        for a, ax in enumerate(self.axes):
            shp = [1] * (2 * naxes)
            shp[2 * a], shp[2 * a + 1] = ax.N, ax.n
            out.append(ax.nodes.reshape(shp))
        return out

    def weights(self, axes=None):
        """Product quadrature weight array over the chosen axes (default all)."""
        naxes = len(self.axes)
        axes = range(naxes) if axes is None else axes
        W = np.ones([1] * (2 * naxes))
        for a in axes:
            shp = [1] * (2 * naxes)
            shp[2 * a], shp[2 * a + 1] = self.axes[a].N, self.axes[a].n
            W = W * self.axes[a].qw.reshape(shp)
        return W
