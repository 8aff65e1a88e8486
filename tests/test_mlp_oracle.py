"""Pins of the FP64 predictor reference: gradients against central finite
differences, closed forms, and descent on a fixed batch."""
from __future__ import annotations

import numpy as np

import synth
from oracle import mlp


def _batch(seed, n=40):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 24))
    y = (rng.random((n, 9)) < 0.3).astype(np.float64)
    m = (rng.random((n, 9)) < 0.8).astype(np.float64)
    return x, y, m


def _params(seed):
    p = synth.mlp_init(seed)
    rng = np.random.default_rng(seed + 1)
    return {k: v.astype(np.float64) + (0.05 * rng.normal(size=v.shape) if k.startswith("b") else 0)
            for k, v in p.items()}


def test_gradients_match_finite_differences():
    p = _params(3)
    x, y, m = _batch(4)
    z, cache = mlp.forward(p, x)
    g = mlp.backward(p, cache, z, y, m)
    rng = np.random.default_rng(0)
    h = 1e-6
    for k in p:
        for _ in range(12):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k][idx] += h
            lp = mlp.loss(mlp.forward(q, x)[0], y, m)
            q[k][idx] -= 2 * h
            lm = mlp.loss(mlp.forward(q, x)[0], y, m)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, g[k][idx])


def test_closed_forms():
    p = {k: np.zeros_like(v, dtype=np.float64) for k, v in synth.mlp_init(1).items()}
    p["b3"] = np.linspace(-2, 2, 9)
    x, y, m = _batch(5)
    z, _ = mlp.forward(p, x)
    assert np.allclose(z, p["b3"][None, :])
    # BCE with constant logits b: mean over mask of softplus(b) - y b
    ref = (m * (np.log1p(np.exp(p["b3"]))[None, :] - y * p["b3"][None, :])).sum() / m.sum()
    assert abs(mlp.loss(z, y, m) - ref) < 1e-12
    # masked-out entries carry no gradient
    g = mlp.backward(p, mlp.forward(p, x)[1], z, y, np.zeros_like(m))
    assert all(np.abs(v).max() == 0 for v in g.values())


def test_descent_on_fixed_batch():
    p = _params(9)
    x, y, m = _batch(6, n=200)
    l0 = mlp.loss(mlp.forward(p, x)[0], y, m)
    st = {}
    for _ in range(50):
        z, c = mlp.forward(p, x)
        p, st = mlp.adam(p, mlp.backward(p, c, z, y, m), st, 1e-2)
    assert mlp.loss(mlp.forward(p, x)[0], y, m) < 0.8 * l0
