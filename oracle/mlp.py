"""FP64 reference of the brick-request predictor network (test
infrastructure; only tests, the smoke check and the bench's CPU-baseline leg
use it).

The predictor is not part of the paper; its definition is this project's:
a 3-layer perceptron 24 -> 64 -> 64 -> 9 with ReLU hidden layers and one
logit per resolution level, trained with binary cross-entropy on the logits
masked per (row, level), mean over the unmasked entries:

    h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), z = h2 W3 + b3
    loss = sum(mask * (softplus(z) - y z)) / sum(mask)

Weights are stored input-major (W1 is 24 x 64).  Plain definitions with
numpy matrix products; no blocking or fusion.
"""
from __future__ import annotations

import numpy as np

SIZES = (24, 64, 64, 9)


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(p: dict, x: np.ndarray):
    x = np.asarray(x, np.float64)
    a1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"] + p["b3"]
    return z, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2)


def loss(z, y, mask) -> float:
    m = np.asarray(mask, np.float64)
    n = m.sum()
    if n == 0:
        return 0.0
    return float((m * (softplus(z) - np.asarray(y, np.float64) * z)).sum() / n)


def backward(p: dict, cache: dict, z, y, mask) -> dict:
    """Gradients of `loss` with respect to every parameter."""
    m = np.asarray(mask, np.float64)
    n = max(m.sum(), 1.0)
    dz = m * (sigmoid(z) - np.asarray(y, np.float64)) / n
    g = {}
    g["W3"] = cache["h2"].T @ dz
    g["b3"] = dz.sum(axis=0)
    dh2 = dz @ p["W3"].T
    da2 = dh2 * (cache["a2"] > 0)
    g["W2"] = cache["h1"].T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"].T
    da1 = dh1 * (cache["a1"] > 0)
    g["W1"] = cache["x"].T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def sgd(p: dict, g: dict, lr: float) -> dict:
    return {k: p[k] - lr * g[k] for k in p}


def adam(p: dict, g: dict, st: dict, lr: float, b1=0.9, b2=0.999, eps=1e-8) -> tuple:
    """One Adam step (Kingma & Ba 2015); st holds m, v and t."""
    t = st.get("t", 0) + 1
    out, m_new, v_new = {}, {}, {}
    for k in p:
        m = b1 * st.get("m", {}).get(k, 0.0) + (1 - b1) * g[k]
        v = b2 * st.get("v", {}).get(k, 0.0) + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
        m_new[k], v_new[k] = m, v
    return out, dict(m=m_new, v=v_new, t=t)
