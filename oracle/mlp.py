"""fp64 reference for the partition-scoring MLP (test infrastructure only).

The learned scheduler is an addition to the paper's method: it scores
partitions in place of the user priority functor of Section 5.2 (the paper's
rule: a partition's priority is the best priority of its buffered
operations).  The network is y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 with
sizes 16 -> 64 -> 64 -> 1, trained with mean squared error.

Flat parameter layout (5,313 values, row-major):
  W1[64,16] | b1[64] | W2[64,64] | b2[64] | W3[1,64] | b3[1]
"""
from __future__ import annotations

import numpy as np

D_IN, H1, H2 = 16, 64, 64
SIZES = [("W1", (H1, D_IN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("W3", (1, H2)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[n], np.float64).ravel() for n, _ in SIZES])


def init(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1])
            p[name] = rng.uniform(-lim, lim, shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def forward(theta, x):
    """Scores [n] for features x [n, 16]; also returns the activations."""
    P = unpack(theta)
    x = np.asarray(x, np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = np.maximum(z2, 0.0)
    y = (a2 @ P["W3"].T + P["b3"])[:, 0]
    return y, (x, z1, a1, z2, a2)


def loss_and_grad(theta, x, target):
    """Mean squared error 1/n sum (y - t)^2 and its gradient (flat, fp64)."""
    P = unpack(theta)
    y, (x, z1, a1, z2, a2) = forward(theta, x)
    n = y.shape[0]
    diff = y - np.asarray(target, np.float64)
    loss = float(np.mean(diff * diff))
    dy = (2.0 / n) * diff[:, None]          # [n,1]
    g = {}
    g["W3"] = dy.T @ a2
    g["b3"] = dy.sum(0)
    da2 = dy @ P["W3"]
    dz2 = da2 * (z2 > 0)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    da1 = dz2 @ P["W2"]
    dz1 = da1 * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015); t counts from 1.  Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
