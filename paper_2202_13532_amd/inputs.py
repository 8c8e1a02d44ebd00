"""Seeded synthetic inputs shared by the library's callers and the tests.

This module holds no arithmetic of the DG method: it evaluates initial
distributions f(x, u, v) on node-coordinate arrays that the caller supplies
(from the library or, in tests, from the oracle), and draws seeded random
numbers.  ``xp`` is the array module (numpy, or torch for device-side
generation of large states); the formulas only use exp/cos/sqrt.

Workloads (sizes and recipes are listed in ``workloads``):
  * landau      -- (1 + eps cos(k x)) exp(-v^2/2)/sqrt(2 pi)           (1D1V)
  * ring        -- exp(-(v_perp - r0)^2 / 2) / Z (1 + eps cos(k x))     (1D2V)
                   Z = 2 pi [exp(-r0^2/2) + r0 sqrt(pi/2)(1 + erf(r0/sqrt 2))]
                   makes the density exactly 1 over the infinite plane.
  * maxwell_multimode -- exp(-(u^2+v^2)/2)/(2 pi) [1 + eps sum_p cos(p k1 x + phi_p)]
                   with phases phi_p ~ U[0, 2 pi) from numpy's default_rng(seed).
  * random_nodal -- U(0, 1) at every node (parity of the linear operator).
  * loss_cone   -- the ring of eq. loss_cone, (s^j e^{-s}) / (2 pi alpha^2 j!),
                   s = v_perp^2 / (2 alpha^2)                           (1D2V)
  * cyclotron_mode -- the linear eigenmode of eq. ic about loss_cone (Sec. 4.1):
                   (f0'(v_perp)/v_perp) Re(psi), psi a 2 nmax + 1 term Bessel
                   sum, for a given root (k, omega) of the dispersion relation.
"""
import math

import numpy as np


def ring_normalisation(r0=3.0):
    return 2.0 * math.pi * (math.exp(-0.5 * r0 * r0)
                            + r0 * math.sqrt(math.pi / 2.0) * (1.0 + math.erf(r0 / math.sqrt(2.0))))


def landau(x, v, k=0.5, eps=0.01, xp=np):
    return (1.0 + eps * xp.cos(k * x)) * xp.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)


def maxwellian_1d(v, vt=1.0, xp=np):
    return xp.exp(-0.5 * (v / vt) ** 2) / (math.sqrt(2.0 * math.pi) * vt)


def maxwellian_2d(u, v, vt=1.0, xp=np):
    return xp.exp(-0.5 * (u * u + v * v) / (vt * vt)) / (2.0 * math.pi * vt * vt)


def ring(u, v, r0=3.0, xp=np):
    vperp = xp.sqrt(u * u + v * v)
    return xp.exp(-0.5 * (vperp - r0) ** 2) / ring_normalisation(r0)


def ring_perturbed(x, u, v, k, eps=1e-3, r0=3.0, xp=np):
    return ring(u, v, r0, xp) * (1.0 + eps * xp.cos(k * x))


def multimode_phases(seed, modes=8):
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, size=modes)


def maxwell_multimode(x, u, v, k1, seed, eps=1e-3, modes=8, xp=np):
    phases = multimode_phases(seed, modes)
    pert = 0.0 * x
    for p in range(1, modes + 1):
        pert = pert + xp.cos(p * k1 * x + float(phases[p - 1]))
    return maxwellian_2d(u, v, 1.0, xp) * (1.0 + eps * pert)


def random_nodal(shape, seed, dtype=np.float64):
    return np.random.default_rng(seed).random(shape).astype(dtype)


def random_field(nx_nodes, seed, scale=0.3):
    """Seeded smooth-ish random electric field values at the x nodes."""
    return scale * np.random.default_rng(seed + 7919).standard_normal(nx_nodes)


def mixture(x, u, v, a, vt, k1, eps=1e-3, r0=3.0, xp=np):
    """a ring(r0) + (1 - a) Maxwellian(vt), times (1 + eps cos(k1 x))."""
    return (a * ring(u, v, r0, xp) + (1.0 - a) * maxwellian_2d(u, v, vt, xp)) * (1.0 + eps * xp.cos(k1 * x))


def loss_cone(u, v, j=6, alpha=1.0, xp=np):
    s = (u * u + v * v) / (2.0 * alpha * alpha)
    return s ** j * xp.exp(-s) / (2.0 * math.pi * alpha * alpha * math.factorial(j))


def cyclotron_mode(x, u, v, kx, k0, omega, j=6, alpha=1.0, nmax=20, sense=-1.0, complex_out=False):
    """Eigenmode of eq. ic for the ring of eq. loss_cone (NumPy, FP64).

    psi = exp(i (kx x + k0 v_perp sin phi)) sum_{|m| <= nmax} m / (m - omega)
    J_m(k0 v_perp) e^{-i m phi};  f1 = (f0'(v_perp) / v_perp) Re(psi), with
    f0'/v_perp = (j - v_perp^2 / (2 alpha^2)) f0 / v_perp^2 (the radial
    gradient of eq. loss_cone).  kx is the wavenumber in units of the x
    coordinate, k0 = kx v_t / omega_c the same wavenumber in inverse Larmor
    radii (the argument of the Bessel functions), omega the root in units of
    the cyclotron frequency.  The angle is phi = atan2(sense v, u): with the
    force F = [u, -E - v B, u B] of this library (B > 0) the gyration runs
    clockwise in (u, v), which the printed mode describes with sense = -1.
    Returns f1 with unit-free amplitude (the caller scales it), or the
    complex (f0'/v_perp) psi when complex_out.
    """
    from scipy import special
    vp = np.sqrt(u * u + v * v)
    vps = np.where(vp > 0.0, vp, 1.0)
    phi = np.arctan2(sense * v, u)
    s = vp * vp / (2.0 * alpha * alpha)
    f0 = s ** j * np.exp(-s) / (2.0 * math.pi * alpha * alpha * math.factorial(j))
    grad = np.where(vp > 0.0, (j - s) * f0 / (vps * vps), 0.0)
    arg = k0 * vp
    acc = np.zeros(np.broadcast(x, u, v).shape, dtype=np.complex128)
    for m in range(-nmax, nmax + 1):
        if m == 0:
            continue
        acc = acc + (m / (m - omega)) * special.jv(m, arg) * np.exp(-1j * m * phi)
    psi = np.exp(1j * (kx * x + k0 * vp * np.sin(phi))) * acc
    return grad * psi if complex_out else grad * psi.real


def broadcast_coords(axes_nodes, xp=np):
    """Reshape per-axis (N, n) node arrays into broadcastable state-layout arrays."""
    naxes = len(axes_nodes)
    out = []
    for a, nodes in enumerate(axes_nodes):
        shp = [1] * (2 * naxes)
        shp[2 * a], shp[2 * a + 1] = nodes.shape[0], nodes.shape[1]
        out.append(nodes.reshape(shp))
    return out


def elliptic_cosine(x, sqrt_m):
    """cn(4 K x | m) (period 1 in x, K the quarter period), the test function
    of the paper's aliasing study (Sec. 5.3.1, errors figure)."""
    from scipy import special
    m = sqrt_m * sqrt_m
    K = special.ellipk(m)
    return special.ellipj(4.0 * K * np.asarray(x, dtype=np.float64), m)[1]
