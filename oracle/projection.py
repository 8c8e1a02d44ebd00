"""L2 projection of a DG function between nested rectilinear grids, FP64.

Test infrastructure (see ``oracle/__init__``).

Used to build training data for the coarse-grid correction: a fine-grid DG
function (nf LGL nodes per element, r fine elements per coarse element) is
projected onto the coarse space (nc LGL nodes per element) axis by axis.  On
one coarse element the coarse nodal values c solve
    M_c c = b,   (M_c)_ij = int l^c_i l^c_j,   b_i = int l^c_i f_fine,
with both integrals evaluated exactly by Gauss-Legendre quadrature (the
integrands are polynomials on every fine sub-element).  The tensor-product
projection applies the one-axis matrix along each axis in turn.

Pinned by tests/test_oracle_projection.py: polynomials of degree < nc are
reproduced exactly, integrals (mass) are preserved, and coarse functions are
fixed points.
"""
import numpy as np

from . import lgl


def projection_matrix(nc, nf, r):
    """P (nc, r*nf): coarse nodal values from the r*nf fine values of one coarse element."""
    xc, _ = lgl.lgl_nodes_weights(nc)
    xf, _ = lgl.lgl_nodes_weights(nf)
    q = nc + nf + 4
    eta, om = np.polynomial.legendre.leggauss(q)
    Mc = np.zeros((nc, nc))
    Bm = np.zeros((nc, r * nf))
    for s in range(r):
        # sub-element s of the reference coarse element [-1, 1]
        a, b = -1.0 + 2.0 * s / r, -1.0 + 2.0 * (s + 1) / r
        x = 0.5 * (a + b) + 0.5 * (b - a) * eta          # coarse reference coordinate
        wq = 0.5 * (b - a) * om
        lc = np.stack([lgl.lagrange_eval(xc, i, x) for i in range(nc)])     # (nc, q)
        lf = np.stack([lgl.lagrange_eval(xf, k, eta) for k in range(nf)])   # (nf, q)
        Mc += (lc * wq) @ lc.T
        Bm[:, s * nf:(s + 1) * nf] = (lc * wq) @ lf.T
    return np.linalg.solve(Mc, Bm)


def project(f_fine, nv, nc, nf, r):
    """Project a fine state [Nf, nf, ...] (1 + nv axes) onto the coarse grid."""
    P = projection_matrix(nc, nf, r)
    out = np.asarray(f_fine, dtype=np.float64)
    naxes = 1 + nv
    for a in range(naxes):
        shp = list(out.shape)
        Nf = shp[2 * a]
        Nc = Nf // r
        # group r fine elements (with their nodes) per coarse element
        x = out.reshape(shp[:2 * a] + [Nc, r * nf] + shp[2 * a + 2:])
        y = np.moveaxis(np.tensordot(x, P, axes=([2 * a + 1], [1])), -1, 2 * a + 1)
        out = y
    return out
