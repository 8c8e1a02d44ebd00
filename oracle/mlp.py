"""FP64 multilayer perceptron: forward, backward, MSE loss and AdamW.

Test infrastructure (see ``oracle/__init__``).

The learned coarse-grid correction is a per-element network: input features
-> three hidden Linear + GELU layers -> Linear output.  GELU is the exact
form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.  Row-major activations:
X is (rows, in), W is (in, out), so y = X W + b.

Pinned by tests/test_oracle_mlp.py: central finite differences of the loss
for every parameter tensor and the input, GELU against its definition and
its derivative by finite differences, AdamW against a hand-expanded first
step and against three steps with different gradients written out with the
moment recurrences unrolled (from the second step on the bias-corrected
moments differ from g and g^2, so the roles of beta1 and beta2 and the
bias-correction exponents are fixed).
"""
import math

import numpy as np
from scipy.special import erf


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * phi


def init_params(sizes, seed):
    """He-style normal init; biases zero.  sizes = [in, h1, ..., out]."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        params.append(rng.standard_normal((a, b)) * math.sqrt(2.0 / a))
        params.append(np.zeros(b))
    return params


def forward(params, X):
    """Returns output and the cache of pre-activations / activations."""
    acts = [np.asarray(X, dtype=np.float64)]
    pres = []
    nl = len(params) // 2
    h = acts[0]
    for l in range(nl):
        z = h @ params[2 * l] + params[2 * l + 1]
        pres.append(z)
        h = gelu(z) if l < nl - 1 else z
        acts.append(h)
    return h, (acts, pres)


def mse(y, target):
    d = y - target
    return float(np.mean(d * d))


def backward(params, cache, y, target):
    """Gradients of mse(y, target) w.r.t. every parameter and the input."""
    acts, pres = cache
    nl = len(params) // 2
    g = 2.0 * (y - target) / y.size
    grads = [None] * len(params)
    for l in reversed(range(nl)):
        if l < nl - 1:
            g = g * gelu_grad(pres[l])
        grads[2 * l] = acts[l].T @ g
        grads[2 * l + 1] = g.sum(axis=0)
        g = g @ params[2 * l].T
    return grads, g


def adamw_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW step (decoupled weight decay on weights only); t counts from 1."""
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        m[i] = b1 * m[i] + (1 - b1) * g
        v[i] = b2 * v[i] + (1 - b2) * g * g
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        decay = wd if i % 2 == 0 else 0.0
        out.append(p - lr * (mh / (np.sqrt(vh) + eps) + decay * p))
    return out
