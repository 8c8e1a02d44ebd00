"""Pins of oracle.harris (Sec. 4.1: eq. harris, eq. loss_cone, eq. transform,
eq. disp) and of the eigenmode initial condition of eq. ic against the
oracle's DG right-hand side."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import grid, harris, lgl, rk
from paper_2202_13532_amd import inputs
from tests.golden import paper_value


@pytest.mark.parametrize("j,alpha", [(6, 1.0), (3, 0.8), (0, 1.3)])
def test_hankel_transform_of_loss_cone_by_quadrature(j, alpha):
    # H0[f](lam) = 2 pi int_0^inf f(v) J0(lam v) v dv, evaluated directly
    for lam in [0.0, 0.4, 1.1, 2.3]:
        val, _ = integrate.quad(lambda v: 2 * math.pi * harris.loss_cone(v, j, alpha) * special.j0(lam * v) * v,
                                0.0, 40.0 * alpha, limit=400, epsabs=1e-14, epsrel=1e-12)
        assert abs(harris.hankel_loss_cone(lam, j, alpha) - val) < 1e-11, (j, alpha, lam)
    # unit density: H0[f0](0) = 1
    assert harris.hankel_loss_cone(0.0, j, alpha) == 1.0


@pytest.mark.parametrize("w", [0.3 + 0.2j, 1.5 + 0.05j, 2.7 - 0.1j, 0.5j])
@pytest.mark.parametrize("k", [0.3, 0.886, 2.5])
def test_maxwellian_equals_bernstein_series(w, k):
    # j = 0 is the Maxwellian; Bernstein's form of the same dispersion function:
    # 1 + (wp/wc)^2 / k^2 [1 - sum_n w / (w - n) I_n(k^2) e^{-k^2}]
    r = 10.0
    series = sum(w / (w - m) * special.ive(m, k * k) for m in range(-80, 81))
    ref = 1.0 + r * r / (k * k) * (1.0 - series)
    got = harris.dispersion(w, k, 0, r, npts=200)
    assert abs(got - ref) < 1e-12 * abs(ref)
    # the paper's 50-point rule is accurate to well below the printed digits
    assert abs(harris.dispersion(w, k, 0, r) - ref) < 1e-6 * abs(ref)


def test_printed_roots():
    g = paper_value("harris_roots")
    for k, wr, wi in g["roots"]:
        w = harris.find_root(k, complex(wr, wi) * 1.02 + 0.01j, g["jring"], g["wp_over_wc"])
        # printed to three decimals
        assert abs(w.real - wr) < 5.01e-4 and abs(w.imag - wi) < 5.01e-4, (k, w)
        assert abs(harris.dispersion(w, k, g["jring"], g["wp_over_wc"])) < 1e-9


def test_fastest_growing_purely_growing_mode_is_near_k0():
    g = paper_value("harris_roots")
    k0 = g["roots"][0][0]
    ks = np.linspace(k0 - 0.05, k0 + 0.05, 21)
    gam = []
    w = 0.35j
    for k in ks:
        w = harris.find_root(k, w, g["jring"], g["wp_over_wc"])
        assert abs(w.real) < 1e-9   # purely growing branch
        gam.append(w.imag)
    kbest = ks[int(np.argmax(gam))]
    assert abs(kbest - k0) <= 0.0051, kbest


@pytest.mark.parametrize("mode", [0, 1])
def test_eigenmode_is_an_eigenfunction_of_the_oracle_rhs(mode):
    """eq. ic about eq. loss_cone grows like exp(-i omega B t) under the DG RHS.

    With F = [u, -E - vB, uB] and B = omega_c/omega_p = 0.1 the linearised
    oracle RHS acting on f1 = (f0'/v_perp) Re(psi) must equal
    Re(-i omega B (f0'/v_perp) psi): checked to the grid's truncation error
    (n = 6, 20 elements per velocity axis on +-8.5)."""
    g0 = paper_value("harris_roots")
    k0, wr, wi = g0["roots"][mode]
    w = harris.find_root(k0, complex(wr, wi), g0["jring"], g0["wp_over_wc"])
    B = 1.0 / g0["wp_over_wc"]
    kx = k0 * B
    n = 6
    g = grid.PhaseGrid(2, n, [6, 20, 20], [0.0, -8.5, -8.5], [2 * math.pi / kx, 8.5, 8.5], B)
    x, u, v = g.coords()
    ops = lgl.operators(n)
    f0 = np.broadcast_to(inputs.loss_cone(u, v, g0["jring"]), g.shape).copy()
    psi = np.broadcast_to(inputs.cyclotron_mode(x, u, v, kx, k0, w, g0["jring"], complex_out=True), g.shape)
    f1 = psi.real
    eps = 1e-6 / np.max(np.abs(f1))
    d = (rk.L(g, ops, f0 + eps * f1) - rk.L(g, ops, f0)) / eps
    expect = (-1j * w * B * psi).real
    assert np.linalg.norm(d - expect) < 0.03 * np.linalg.norm(expect)


@pytest.mark.parametrize("which", ["A", "B"])
def test_case_study_density_amplitude_of_the_mode(which):
    """The closed form (Jacobi-Anger) of the mode's density used to scale the
    case-study perturbation equals brute-force quadrature of eq. ic over the
    velocity plane; the ring's thermal energy is App. B's exact moment."""
    from paper_2202_13532_amd import case_study as cs
    kx, k0, _, hi = cs.geometry(which)
    om = cs.CASES[which]["omega"]
    h = 0.03
    g = np.arange(-12 + h / 2, 12, h)
    psi = inputs.cyclotron_mode(0.0, g[:, None], g[None, :], kx, k0, om, 6, complex_out=True)
    brute = psi.sum() * h * h
    assert abs(cs.mode_density(k0, om) - brute) < 1e-10 * abs(brute)
    # App. B: alpha^2 (j + 1 - (Gamma(j + 3/2) / Gamma(j + 1))^2), close to 1/4 for large j
    per_length = cs.thermal_energy(which) / hi[0]
    assert abs(per_length - (7.0 - (special.gamma(7.5) / special.gamma(7.0)) ** 2)) < 1e-12
    assert abs(per_length / paper_value("ring_thermal_energy_per_length")["value"] - 1.0) < 0.03
