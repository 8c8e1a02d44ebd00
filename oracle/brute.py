"""Dense brute-force assembly of the DG weak form on tiny grids, FP64.

Test infrastructure (see ``oracle/__init__``); used only to pin ``oracle.rhs``.

Instead of the paper's one-dimensional closed-form operators and the
tensor-product decoupling (eq. decoupled), this module evaluates the weak form
(eq. part_2 integrated by parts once, eq. weak before multiplying by M^-1)
element by element with full d-dimensional Gauss-Legendre quadrature:

    sum_b M_gb du_b/dt = sum_j int_elem F_j(x) d_j L_g(x) dx
                         - sum_faces n_j int_face Fnum(y) L_g(y) dS,

where L_b is the d-dimensional tensor-product Lagrange basis (eq. d_dim_lagrange),
the flux is its nodal interpolant F_j(x) = sum_b a_j(x_b) u_b L_b(x) as in the
method, Fnum is the upwind face flux interpolated on the face nodes, and M is
integrated by quadrature and inverted with a dense solve.  Only the LGL node
positions and the Lagrange product formula are shared with ``oracle.lgl``.
It is O((n^d)^2 q^d) per element, so only grids of a few elements are usable.
"""
import itertools

import numpy as np

from . import lgl


def _lagrange_deriv_eval(xi, j, x):
    """l'_j(x) by differentiating the product formula term by term."""
    n = len(xi)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for m in range(n):
        if m == j:
            continue
        term = np.full_like(x, 1.0 / (xi[j] - xi[m]))
        for k in range(n):
            if k != j and k != m:
                term = term * (x - xi[k]) / (xi[j] - xi[k])
        out += term
    return out


def brute_rhs(grid, f, E):
    """Same quantity as oracle.rhs.rhs, assembled densely element by element."""
    naxes = len(grid.axes)
    n = grid.n
    xi, _ = lgl.lgl_nodes_weights(n)
    q = n + 4
    eta, om = np.polynomial.legendre.leggauss(q)
    phi = np.stack([lgl.lagrange_eval(xi, j, eta) for j in range(n)], axis=1)        # (q, n)
    dphi = np.stack([_lagrange_deriv_eval(xi, j, eta) for j in range(n)], axis=1)    # (q, n)
    d = naxes
    nb = n ** d
    nodes_md = list(itertools.product(range(n), repeat=d))      # basis multi-indices
    quad_md = list(itertools.product(range(q), repeat=d))
    # basis values / derivatives at volume quadrature points
    Bv = np.zeros((len(quad_md), nb))
    Gv = np.zeros((d, len(quad_md), nb))
    wq = np.zeros(len(quad_md))
    for iq, Q in enumerate(quad_md):
        wq[iq] = np.prod([om[Q[a]] for a in range(d)])
        for ib, b in enumerate(nodes_md):
            vals = [phi[Q[a], b[a]] for a in range(d)]
            Bv[iq, ib] = np.prod(vals)
            for j in range(d):
                dv = list(vals)
                dv[j] = dphi[Q[j], b[j]]
                Gv[j, iq, ib] = np.prod(dv)
    Nel = [ax.N for ax in grid.axes]
    half = [ax.dx / 2.0 for ax in grid.axes]
    vol = np.prod(half)
    M = vol * (Bv.T * wq) @ Bv
    Minv = np.linalg.inv(M)
    E = np.asarray(E, dtype=np.float64).reshape(grid.axes[0].N, n)
    B = grid.omega_c

    def speed(j, elem, node):
        # physical coordinates of a node, eq. vlasov speeds
        c = [grid.axes[a].nodes[elem[a], node[a]] for a in range(d)]
        if d == 2:
            return c[1] if j == 0 else -E[elem[0], node[0]]
        if j == 0:
            return c[1]
        if j == 1:
            return -E[elem[0], node[0]] - c[2] * B
        return c[1] * B

    def block(elem):
        sl = []
        for a in range(d):
            sl += [elem[a], slice(None)]
        return f[tuple(sl)].reshape(-1)

    out = np.zeros_like(f, dtype=np.float64)
    for elem in itertools.product(*[range(N) for N in Nel]):
        u = block(elem)
        rhs_vec = np.zeros(nb)
        for j in range(d):
            Jj = 2.0 / grid.axes[j].dx
            Fn = np.array([speed(j, elem, b) * u[ib] for ib, b in enumerate(nodes_md)])
            # volume term  int F_j d_j L_g dx
            Fq = Bv @ Fn
            rhs_vec += Jj * vol * (Gv[j].T * wq) @ Fq
            # face terms on the two faces of axis j
            others = [a for a in range(d) if a != j]
            face_md = list(itertools.product(range(n), repeat=d - 1))
            fq_md = list(itertools.product(range(q), repeat=d - 1))
            dS = np.prod([half[a] for a in others])
            periodic = (j == 0) or grid.vbc == "periodic"
            for side, normal in ((0, -1.0), (n - 1, +1.0)):
                nb_elem = list(elem)
                nb_elem[j] += 1 if side == n - 1 else -1
                outside = nb_elem[j] < 0 or nb_elem[j] >= Nel[j]
                nb_elem[j] %= Nel[j]
                ub = block(tuple(nb_elem))
                Fstar = np.zeros(len(face_md))
                for iface, fn in enumerate(face_md):
                    own = [0] * d
                    nbn = [0] * d
                    for k, a in enumerate(others):
                        own[a] = fn[k]
                        nbn[a] = fn[k]
                    own[j] = side
                    nbn[j] = (n - 1) - side
                    a_s = speed(j, elem, own)
                    own_val = a_s * u[nodes_md.index(tuple(own))]
                    if outside and not periodic:
                        nbr_val = 0.0
                    else:
                        nbr_val = speed(j, tuple(nb_elem), nbn) * ub[nodes_md.index(tuple(nbn))]
                    upwind_own = (a_s > 0) if side == n - 1 else (a_s < 0)
                    if a_s == 0:
                        Fstar[iface] = 0.0
                    else:
                        Fstar[iface] = own_val if upwind_own else nbr_val
                # integrate Fstar(y) L_g(y) over the face
                for ifq, Qf in enumerate(fq_md):
                    wf = np.prod([om[Qf[k]] for k in range(d - 1)])
                    fval = 0.0
                    for iface, fn in enumerate(face_md):
                        fval += Fstar[iface] * np.prod([phi[Qf[k], fn[k]] for k in range(d - 1)])
                    for ig, g in enumerate(nodes_md):
                        if g[j] != side:
                            continue        # l_g(+-1) is zero unless g_j is that end node
                        lg = np.prod([phi[Qf[k], g[a]] for k, a in enumerate(others)])
                        rhs_vec[ig] -= normal * wf * dS * fval * lg
        du = Minv @ rhs_vec
        sl = []
        for a in range(d):
            sl += [elem[a], slice(None)]
        out[tuple(sl)] = du.reshape([n] * d)
    return out
