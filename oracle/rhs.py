"""Weak-form DG semi-discrete right-hand side of the Vlasov equation, FP64.

Test infrastructure (see ``oracle/__init__``).

The Vlasov equation is the conservation law d_t f + d_j (F^j f) = 0 with the
phase-space speeds of eq. vlasov (the flow is divergence free, so the
advective and conservative forms agree):
    1D2V, axes (x, u, v):  F = [u,  dPhi/dx - v B,  u B] = [u, -E - v B, u B]
    1D1V, axes (x, v):     F = [v,  -E]                   (B = 0, one velocity)
with E = -dPhi/dx the electric field at the x nodes.

Per element the weak form (eq. weak) reads du/dt = Upsilon F - Xi Fnum.  On
a tensor-product grid it decouples into one contraction per axis along that
axis's node index (eq. internal_flux, eq. decoupled) and one face product per
axis (eq. numerical_flux), each scaled by the axis Jacobian J = 2/dx (Sec. 2).
The numerical flux is upwind (Sec. 3.1.1) and is assembled as in App. A: with
[a>0] and [a<0] the sign selectors, on the left face (outward normal -1)
    Fnum_L = -( roll(F_R, +1) [a>0] + F_L [a<0] )
and on the right face (outward normal +1)
    Fnum_R =    F_R [a>0] + roll(F_L, -1) [a<0],
where F_L, F_R are the element's own first/last node values and roll brings in
the neighbouring element's value.  Every axis is periodic (App. A rolls every
axis); ``vbc="zero_inflow"`` instead makes the value beyond a velocity-axis
edge zero.

Pinned by tests/test_oracle_rhs.py: dense brute-force weak-form assembly by
quadrature on tiny grids (oracle.brute), discrete mass conservation, exact
free streaming and gyration, and the Landau damping rate.
"""
import numpy as np


def _take(arr, axis, idx):
    sl = [slice(None)] * arr.ndim
    sl[axis] = idx
    return arr[tuple(sl)]


def _roll_faces(face, elem_axis, shift, periodic):
    """Neighbouring element's face value; zero beyond the edge if not periodic."""
    out = np.roll(face, shift, axis=elem_axis)
    if not periodic:
        sl = [slice(None)] * out.ndim
        sl[elem_axis] = 0 if shift > 0 else -1
        out[tuple(sl)] = 0.0
    return out


def axis_term(F, speed, a, ax, ops, periodic=True):
    """J_a (Upsilon F - Xi Fnum) along axis a for the flux array F = speed * f.

    ``speed`` is broadcastable to F and constant along axis a (it depends only
    on the other coordinates), so its sign selects the upwind side.
    """
    ndim = F.ndim
    ea, na = 2 * a, 2 * a + 1                   # element axis, node axis
    ups, xi = ops["Ups"], ops["Xi"]
    n = ups.shape[0]
    # internal flux product, contraction along the node index of axis a
    vol = np.moveaxis(np.tensordot(F, ups, axes=([na], [1])), -1, na)
    # face values of F and the speed sign (speed does not vary along axis a)
    F_L = _take(F, na, 0)
    F_R = _take(F, na, n - 1)
    s = np.broadcast_to(speed, F.shape)
    s_face = _take(s, na, 0)
    pos = (s_face > 0).astype(np.float64)
    neg = (s_face < 0).astype(np.float64)
    ea_face = ea                               # node axis removed lies after ea
    nf_left = -(_roll_faces(F_R, ea_face, +1, periodic) * pos + F_L * neg)
    nf_right = F_R * pos + _roll_faces(F_L, ea_face, -1, periodic) * neg
    num_flux = np.stack([nf_left, nf_right], axis=na)      # size 2 at node axis
    surf = np.moveaxis(np.tensordot(num_flux, xi, axes=([na], [1])), -1, na)
    assert surf.ndim == ndim
    return ax.J * (vol - surf)


def speeds(grid, E):
    """Phase-space speed arrays (broadcastable to the state) of eq. vlasov."""
    E = np.asarray(E, dtype=np.float64)
    if grid.nv == 1:
        x, v = grid.coords()
        Ex = E.reshape(grid.axes[0].N, grid.n, 1, 1)
        return [v, -Ex]
    x, u, v = grid.coords()
    Ex = E.reshape(grid.axes[0].N, grid.n, 1, 1, 1, 1)
    B = grid.omega_c
    return [u, -Ex - v * B, u * B]


def rhs(grid, ops, f, E):
    """Full semi-discrete RHS L(f) for the given field E at the x nodes."""
    f = np.asarray(f, dtype=np.float64)
    sp = speeds(grid, E)
    out = np.zeros_like(f)
    for a, ax in enumerate(grid.axes):
        periodic = (a == 0) or grid.vbc == "periodic"
        F = sp[a] * f
        out += axis_term(F, sp[a], a, ax, ops, periodic)
    return out


def density(grid, f):
    """n_mj = int f dv at the x nodes by velocity LGL quadrature (eq. poisson)."""
    W = grid.weights(axes=range(1, len(grid.axes)))
    naxes = len(grid.axes)
    return np.sum(f * W, axis=tuple(range(2, 2 * naxes)))
