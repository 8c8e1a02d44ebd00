"""Pins of oracle.mlp (finite differences, GELU definition, AdamW) and
oracle.projection (exact polynomials, mass, fixed points)."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import grid, mlp, projection


def test_gelu_definition_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x), x * 0.5 * (1 + erf(x / math.sqrt(2))), atol=0, rtol=0)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15   # Phi(1)


def test_mlp_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 5, 6, 4, 3]
    params = mlp.init_params(sizes, 1)
    params = [p + 0.1 * rng.standard_normal(p.shape) for p in params]
    X = rng.standard_normal((9, 7))
    T = rng.standard_normal((9, 3))
    y, cache = mlp.forward(params, X)
    grads, gX = mlp.backward(params, cache, y, T)
    h = 1e-6
    for i, p in enumerate(params):
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            pp = [q.copy() for q in params]
            pm = [q.copy() for q in params]
            pp[i][idx] += h
            pm[i][idx] -= h
            fd = (mlp.mse(mlp.forward(pp, X)[0], T) - mlp.mse(mlp.forward(pm, X)[0], T)) / (2 * h)
            assert abs(fd - grads[i][idx]) < 1e-7 * max(1.0, abs(fd)), (i, idx)
    for idx in [(0, 0), (3, 4), (8, 6)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        fd = (mlp.mse(mlp.forward(params, Xp)[0], T) - mlp.mse(mlp.forward(params, Xm)[0], T)) / (2 * h)
        assert abs(fd - gX[idx]) < 1e-7


def test_adamw_first_step():
    p = [np.array([[1.0, -2.0]]), np.array([0.5])]
    g = [np.array([[0.1, -0.3]]), np.array([2.0])]
    m = [np.zeros_like(x) for x in p]
    v = [np.zeros_like(x) for x in p]
    out = mlp.adamw_step(p, g, m, v, 1, lr=0.01, wd=0.1)
    # first step: m_hat = g, v_hat = g^2 -> update = sign(g) (up to eps) + wd * w on weights
    exp_w = p[0] - 0.01 * (g[0] / (np.abs(g[0]) + 1e-8) + 0.1 * p[0])
    exp_b = p[1] - 0.01 * (g[1] / (np.abs(g[1]) + 1e-8))
    assert np.allclose(out[0], exp_w, atol=1e-15) and np.allclose(out[1], exp_b, atol=1e-15)


def test_adamw_three_steps_hand_expanded():
    # Three steps with different gradients, written out with the moment
    # recurrences unrolled: m_t = (1-b1) sum_s b1^(t-s) g_s and
    # v_t = (1-b2) sum_s b2^(t-s) g_s^2, bias-corrected by 1 - b^t.  From t = 2
    # on m_hat != g and v_hat != g^2, so a swapped b1/b2, a wrong exponent in
    # the bias correction or decay on the bias term changes the result.
    b1, b2, eps, lr, wd = 0.9, 0.999, 1e-8, 0.05, 0.2
    w0, c0 = np.array([[0.7, -1.1, 0.25]]), np.array([0.3])
    gw = [np.array([[0.5, -0.2, 1.0]]), np.array([[-0.3, 0.4, 0.1]]), np.array([[0.2, 0.2, -0.6]])]
    gb = [np.array([1.5]), np.array([-0.5]), np.array([0.25])]
    params = [w0.copy(), c0.copy()]
    m = [np.zeros_like(w0), np.zeros_like(c0)]
    v = [np.zeros_like(w0), np.zeros_like(c0)]
    for t in (1, 2, 3):
        params = mlp.adamw_step(params, [gw[t - 1], gb[t - 1]], m, v, t, lr=lr, b1=b1, b2=b2, eps=eps, wd=wd)
    # hand expansion
    w, c = w0.copy(), c0.copy()
    for t in (1, 2, 3):
        mw = (1 - b1) * sum(b1 ** (t - s) * gw[s - 1] for s in range(1, t + 1))
        vw = (1 - b2) * sum(b2 ** (t - s) * gw[s - 1] ** 2 for s in range(1, t + 1))
        mb = (1 - b1) * sum(b1 ** (t - s) * gb[s - 1] for s in range(1, t + 1))
        vb = (1 - b2) * sum(b2 ** (t - s) * gb[s - 1] ** 2 for s in range(1, t + 1))
        w = w - lr * ((mw / (1 - b1 ** t)) / (np.sqrt(vw / (1 - b2 ** t)) + eps) + wd * w)
        c = c - lr * ((mb / (1 - b1 ** t)) / (np.sqrt(vb / (1 - b2 ** t)) + eps))
    assert np.max(np.abs(params[0] - w)) < 1e-14 and np.max(np.abs(params[1] - c)) < 1e-14
    # the step-2 bias term, worked by hand: m = 0.09*1.5 + 0.1*(-0.5) = 0.085,
    # v = 0.999*0.001*2.25 + 0.001*0.25 = 0.00249775; m_hat = 0.085/0.19,
    # v_hat = 0.00249775/0.001999
    p2 = [w0.copy(), c0.copy()]
    m2 = [np.zeros_like(w0), np.zeros_like(c0)]
    v2 = [np.zeros_like(w0), np.zeros_like(c0)]
    for t in (1, 2):
        p2 = mlp.adamw_step(p2, [gw[t - 1], gb[t - 1]], m2, v2, t, lr=lr, b1=b1, b2=b2, eps=eps, wd=wd)
    assert abs(m2[1][0] - 0.085) < 1e-15 and abs(v2[1][0] - 0.00249775) < 1e-15
    step1 = 1.5 / (1.5 + eps)
    step2 = (0.085 / 0.19) / (math.sqrt(0.00249775 / 0.001999) + eps)
    assert abs(p2[1][0] - (0.3 - lr * step1 - lr * step2)) < 1e-14


@pytest.mark.parametrize("nc,nf,r", [(4, 8, 2), (3, 5, 3), (4, 4, 2), (2, 6, 4)])
def test_projection_exact_on_coarse_polynomials(nc, nf, r):
    # f = polynomial of degree nc-1 in x on each coarse element is reproduced exactly
    Nc = 3
    fine = grid.Axis(0.0, 3.0, Nc * r, nf)
    coarse = grid.Axis(0.0, 3.0, Nc, nc)
    poly = np.polynomial.Polynomial(np.arange(1, nc + 1) * 0.3)
    fvals = poly(fine.nodes)
    P = projection.project(fvals, 0, nc, nf, r)
    assert np.max(np.abs(P - poly(coarse.nodes))) < 1e-12


@pytest.mark.parametrize("nc,nf,r", [(4, 8, 2), (3, 7, 2)])
def test_projection_preserves_mass_and_fixes_coarse_functions(nc, nf, r):
    rng = np.random.default_rng(nc + nf)
    Nc = (2, 3, 2)
    fine = grid.PhaseGrid(2, nf, [Nc[0] * r, Nc[1] * r, Nc[2] * r], [0, -1, -2], [1, 2, 2])
    coarse = grid.PhaseGrid(2, nc, list(Nc), [0, -1, -2], [1, 2, 2])
    f = rng.random(fine.shape)
    Pf = projection.project(f, 2, nc, nf, r)
    assert Pf.shape == coarse.shape
    assert abs(np.sum(coarse.weights() * Pf) - np.sum(fine.weights() * f)) < 1e-12 * np.sum(fine.weights() * f)
    # a coarse-grid function sampled on the fine nodes projects back to itself
    x, u, v = coarse.coords()
    g = np.broadcast_to(np.sin(2 * x) * np.cos(u) + v, coarse.shape)
    # evaluate the coarse interpolant at the fine nodes (per axis Lagrange evaluation)
    from oracle import lgl
    xc, _ = lgl.lgl_nodes_weights(nc)
    xf, _ = lgl.lgl_nodes_weights(nf)
    E = np.zeros((r * nf, nc))
    for s in range(r):
        a, b = -1 + 2 * s / r, -1 + 2 * (s + 1) / r
        xs = 0.5 * (a + b) + 0.5 * (b - a) * xf
        for i in range(nc):
            E[s * nf:(s + 1) * nf, i] = lgl.lagrange_eval(xc, i, xs)
    h = np.asarray(g, dtype=np.float64)
    for ax in range(3):
        shp = list(h.shape)
        y = np.moveaxis(np.tensordot(h, E, axes=([2 * ax + 1], [1])), -1, 2 * ax + 1)
        shp2 = list(y.shape)
        h = y.reshape(shp2[:2 * ax] + [shp2[2 * ax] * r, nf] + shp2[2 * ax + 2:])
    back = projection.project(h, 2, nc, nf, r)
    assert np.max(np.abs(back - g)) < 1e-12
