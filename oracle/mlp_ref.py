"""CPU reference of the algorithm selector's network, in float64.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the GPU kernels' forward
pass, gradient and Adam step.  Nothing in the library imports it.

The network is a plain multilayer perceptron 4 -> 64 -> 64 -> 5 with ReLU
hidden layers on normalised inputs z = (x - mean) / std; its loss is the
squared error over the finite targets, L = scale * sum (y - t)^2.  The
gradient is written out by the chain rule, layer by layer (backpropagation),
and pinned in tests by central finite differences of ``loss``.  The Adam step
follows Kingma & Ba (2015), Algorithm 1, with the bias-corrected moments, and
an optional cosine decay of the step size.
"""
from __future__ import annotations

import numpy as np

IN, H, OUT = 4, 64, 5
LAYOUT = (("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)),
          ("b3", (OUT,)))
NPARAMS = sum(int(np.prod(s)) for _, s in LAYOUT)


def unpack(p: np.ndarray) -> dict:
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in LAYOUT:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    assert o == NPARAMS == p.size
    return out


def pack(w: dict) -> np.ndarray:
    return np.concatenate([np.asarray(w[name], dtype=np.float64).ravel() for name, _ in LAYOUT])


def forward(p, norm, x):
    """Outputs y[B][OUT] and the activations the gradient needs."""
    w = unpack(p)
    norm = np.asarray(norm, dtype=np.float64)
    z = (np.asarray(x, dtype=np.float64) - norm[:IN]) / norm[IN:]
    a1 = z @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w["W3"].T + w["b3"]
    return y, (z, a1, h1, a2, h2)


def loss(p, norm, x, t, scale) -> float:
    y, _ = forward(p, norm, x)
    t = np.asarray(t, dtype=np.float64)
    ok = ~np.isnan(t)
    e = np.where(ok, y - np.where(ok, t, 0.0), 0.0)
    return float(scale * np.sum(e * e))


def grad(p, norm, x, t, scale) -> np.ndarray:
    """dL/dp by backpropagation (flat, in the parameter layout)."""
    w = unpack(p)
    y, (z, a1, h1, a2, h2) = forward(p, norm, x)
    t = np.asarray(t, dtype=np.float64)
    ok = ~np.isnan(t)
    dy = np.where(ok, 2.0 * scale * (y - np.where(ok, t, 0.0)), 0.0)   # dL/dy
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    da2 = (dy @ w["W3"]) * (a2 > 0)                                    # through ReLU
    g["W2"], g["b2"] = da2.T @ h1, da2.sum(axis=0)
    da1 = (da2 @ w["W2"]) * (a1 > 0)
    g["W1"], g["b1"] = da1.T @ z, da1.sum(axis=0)
    return pack(g)


def numeric_grad(p, norm, x, t, scale, idx, h=1e-6) -> np.ndarray:
    """Central differences of ``loss`` for the parameters listed in idx."""
    p = np.asarray(p, dtype=np.float64)
    out = np.empty(len(idx))
    for k, i in enumerate(idx):
        q = p.copy()
        q[i] += h
        lp = loss(q, norm, x, t, scale)
        q[i] -= 2 * h
        lm = loss(q, norm, x, t, scale)
        out[k] = (lp - lm) / (2 * h)
    return out


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, total_steps=0):
    """One Adam step at step number `step` (1-based, per parameter array).
    Returns (p, m, v)."""
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    rate = lr
    if total_steps > 0:
        rate = lr * 0.5 * (1 + np.cos(np.pi * min(step, total_steps) / total_steps))
    return p - rate * mhat / (np.sqrt(vhat) + eps), m, v
