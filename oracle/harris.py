"""Harris dispersion relation of the loss-cone (ring) distribution, FP64.

Test infrastructure (see ``oracle/__init__``).

Sec. 4.1: linearising the magnetised Vlasov-Poisson system about cyclotron
orbits and Fourier transforming in x and t gives the dispersion function in
its integral form (eq. harris),

    eps(w, k) = 1 + (wp/wc)^2 / sin(pi w) int_0^pi sin(theta) sin(w theta)
                    H0[f0](2 k cos(theta/2)) dtheta,

with w in units of the cyclotron frequency and k in inverse Larmor radii.  For
the ring f0 of eq. loss_cone (parameter j, thermal speed alpha) the
zero-order Hankel transform is a Laguerre polynomial times a Gaussian
(eq. transform): H0[f0](lam) = L_j(alpha^2 lam^2 / 2) exp(-alpha^2 lam^2 / 2),
so with beta = alpha^2 lam^2 / 2 = 2 alpha^2 k^2 cos^2(theta/2) the integrand
of eq. disp is sin(w theta) sin(theta) L_j(beta) e^{-beta}.  The paper
evaluates the theta integral with a 50-point Gauss-Legendre rule; so does
``dispersion`` by default.

Pinned by tests/test_oracle_harris.py:
  * the Hankel transform against direct quadrature of eq. loss_cone
    (2 pi int f0(v) J0(lam v) v dv);
  * for j = 0 (Maxwellian) the dispersion function equals Bernstein's series
    1 + (wp/wc)^2 / k^2 (1 - sum_n w/(w - n) I_n(k^2) e^{-k^2}), a textbook
    closed form reached by a different route;
  * the two roots the paper prints for j = 6, wp/wc = 10: (k, w) = (0.886,
    0.349i) (the fastest-growing purely growing mode) and (1.4, 1.182 +
    0.131i).
"""
import math

import numpy as np
from scipy import special


def hankel_loss_cone(lam, j, alpha=1.0):
    """H0[f0](lam) of the ring distribution of eq. loss_cone (eq. transform)."""
    b = 0.5 * alpha * alpha * np.asarray(lam, dtype=np.float64) ** 2
    return special.eval_laguerre(j, b) * np.exp(-b)


def loss_cone(vperp, j, alpha=1.0):
    """Ring distribution f0(v_perp) of eq. loss_cone, normalised to unit density."""
    s = np.asarray(vperp, dtype=np.float64) ** 2 / (2.0 * alpha * alpha)
    return s ** j * np.exp(-s) / (2.0 * math.pi * alpha * alpha * math.factorial(j))


def dispersion(w, k, j, wp_over_wc, alpha=1.0, npts=50):
    """eps(w, k) of eq. disp by npts-point Gauss-Legendre quadrature on [0, pi]."""
    x, q = np.polynomial.legendre.leggauss(npts)
    theta = 0.5 * math.pi * (x + 1.0)
    q = 0.5 * math.pi * q
    lam = 2.0 * k * np.cos(0.5 * theta)
    integral = np.sum(q * np.sin(w * theta) * np.sin(theta) * hankel_loss_cone(lam, j, alpha))
    return 1.0 + wp_over_wc ** 2 * integral / np.sin(math.pi * w)


def find_root(k, w_guess, j, wp_over_wc, alpha=1.0, npts=50, tol=1e-13, maxit=100):
    """A root w of eps(., k) near w_guess by the secant iteration."""
    w0 = complex(w_guess)
    w1 = w0 * (1.0 + 1e-3) + 1e-4
    f0 = dispersion(w0, k, j, wp_over_wc, alpha, npts)
    f1 = dispersion(w1, k, j, wp_over_wc, alpha, npts)
    for _ in range(maxit):
        w2 = w1 - f1 * (w1 - w0) / (f1 - f0)
        w0, f0 = w1, f1
        w1 = w2
        f1 = dispersion(w1, k, j, wp_over_wc, alpha, npts)
        if abs(w1 - w0) < tol * max(1.0, abs(w1)):
            return w1
    raise RuntimeError("secant iteration did not converge")
