"""Learned lookup tables: POD basis and a small MLP (oracle, test infrastructure only).

Not part of the paper, which precomputes one table per reference tile
(Section 3.1.1, 3.2.3).  For a parameterised tile family the table T(p) is
approximated by  T(p) ~ Tbar + Phi c(p):
  * POD: Tbar = mean of the snapshot tables, Phi = leading r left singular
    vectors of the centred snapshot matrix X (via the eigenpairs of the Gram
    matrix X^T X), sigma = singular values;
  * MLP: x -> GELU(x W1 + b1) -> GELU(. W2 + b2) -> . W3 + b3, GELU(z) =
    z Phi_N(z) = 0.5 z (1 + erf(z / sqrt 2)), mean-squared-error loss
    L = mean((y - target)^2) over batch and outputs, trained with Adam.
Everything in float64 with hand-written backpropagation; it is the gradient
reference for the GPU kernels.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def pod(snapshots: np.ndarray, r: int):
    """snapshots (n_s, n_entries) -> (mean (n_entries,), basis (n_entries, r), sigma (n_s,) all values)."""
    X = np.asarray(snapshots, dtype=np.float64)
    mean = X.mean(axis=0)
    Xc = (X - mean).T                      # (n_entries, n_s)
    G = Xc.T @ Xc
    lam, V = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    lam, V = np.clip(lam[order], 0.0, None), V[:, order]
    sigma = np.sqrt(lam)
    basis = Xc @ V[:, :r] / sigma[None, :r]
    return mean, basis, sigma


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_mlp(widths, seed: int):
    """Weights W_l (in, out) ~ U(-1/sqrt(in), 1/sqrt(in)), biases zero."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(widths[:-1], widths[1:]):
        bound = 1.0 / math.sqrt(fi)
        params.append(rng.uniform(-bound, bound, size=(fi, fo)))
        params.append(np.zeros(fo))
    return params


def mlp_forward(params, x):
    """Returns output and the cache of pre-activations (for backprop)."""
    n_layers = len(params) // 2
    h = x
    cache = [x]
    for l in range(n_layers):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W + b
        cache.append(z)
        h = gelu(z) if l < n_layers - 1 else z
    return h, cache


def mse_loss(y, target):
    return float(np.mean((y - target) ** 2))


def mlp_backward(params, cache, dy):
    """Gradients of the loss w.r.t. every parameter given dL/dy."""
    n_layers = len(params) // 2
    grads = [None] * len(params)
    g = dy
    for l in reversed(range(n_layers)):
        z = cache[l + 1]
        if l < n_layers - 1:
            g = g * gelu_grad(z)
        h_in = cache[0] if l == 0 else gelu(cache[l])
        grads[2 * l] = h_in.T @ g
        grads[2 * l + 1] = g.sum(axis=0)
        g = g @ params[2 * l].T
    return grads


def loss_and_grads(params, x, target):
    y, cache = mlp_forward(params, x)
    dy = 2.0 * (y - target) / y.size
    return mse_loss(y, target), mlp_backward(params, cache, dy)


def adam_update(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), in place on p, m, v."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    p -= lr * mhat / (np.sqrt(vhat) + eps)
