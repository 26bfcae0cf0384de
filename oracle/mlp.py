"""FP64 reference of the warm-start network: a 3-layer perceptron
x -> relu(x W1 + b1) -> relu(. W2 + b2) -> . W3 + b3, its mean-squared-error
loss, the analytic backward pass, and one Adam step.

The paper has no learned component; this network is an addition on top of the
method (its output only seeds the fixed-point iteration, which still runs to
tolerance).  The gradients are pinned by central finite differences in the
tests; the training outcome itself is measured, not pinned (parity unpinned
for the learned gain).  Weights are stored [fan_in, fan_out], row-major.
"""
from __future__ import annotations

import numpy as np


def init_params(sizes, seed: int):
    """He-uniform weights, zero biases, in FP64."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / fi)
        params.append(rng.uniform(-lim, lim, size=(fi, fo)))
        params.append(np.zeros(fo))
    return params


def forward(params, x):
    """Returns (y, cache) for params [W1,b1,W2,b2,W3,b3]."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def mse(y, t) -> float:
    """Loss = sum (y - t)^2 / (rows * cols)."""
    d = y - t
    return float(np.sum(d * d) / d.size)


def backward(params, cache, y, t):
    """Gradients [dW1,db1,dW2,db2,dW3,db3] of mse(y, t)."""
    W1, b1, W2, b2, W3, b3 = params
    x, z1, h1, z2, h2 = cache
    dy = 2.0 * (y - t) / y.size
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0.0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0.0)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update (Kingma & Ba 2015, bias-corrected); ``step`` starts at 1."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= b1
        mm += (1.0 - b1) * g
        vv *= b2
        vv += (1.0 - b2) * g * g
        mhat = mm / (1.0 - b1 ** step)
        vhat = vv / (1.0 - b2 ** step)
        p -= lr * mhat / (np.sqrt(vhat) + eps)
