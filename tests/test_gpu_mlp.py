"""The predictor's MFMA kernels against the FP64 reference: forward logits,
gradients and Adam steps (FP16 operands, FP32 accumulation)."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_04393_amd import resoct  # noqa: E402


def _data(seed, rows):
    rng = np.random.default_rng(seed)
    x = np.zeros((rows, 32), np.float16)
    x[:, :24] = rng.normal(size=(rows, 24)).astype(np.float16)
    y = np.zeros((rows, 16), np.uint8)
    m = np.zeros((rows, 16), np.uint8)
    y[:, :9] = rng.random((rows, 9)) < 0.3
    m[:, :9] = rng.random((rows, 9)) < 0.85
    return x, y, m


def _params(seed):
    p = synth.mlp_init(seed)
    rng = np.random.default_rng(seed + 11)
    for k in ("b1", "b2", "b3"):
        p[k] = (0.1 * rng.normal(size=p[k].shape)).astype(np.float32)
    return p


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _relerr(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("rows", [1, 37, 1000, 32768])
def test_forward_matches_reference(rows):
    x, y, m = _data(1, rows)
    p = _params(2)
    net = resoct.Mlp()
    net.set_weights(p)
    z = net.forward(_dev(x)).cpu().numpy()[:, :9]
    zr, _ = ref.forward({k: v.astype(np.float64) for k, v in p.items()}, x[:, :24].astype(np.float64))
    err = np.abs(z - zr).max() / max(np.abs(zr).max(), 1e-6)
    print(f"[mlp-forward rows={rows}] max rel err {err:.2e}")
    assert err <= 1e-2


def test_gradients_match_reference():
    x, y, m = _data(3, 4099)
    p = _params(4)
    net = resoct.Mlp()
    net.set_weights(p)
    g, loss = net.gradients(_dev(x), _dev(y), _dev(m))
    pd = {k: v.astype(np.float64) for k, v in p.items()}
    z, cache = ref.forward(pd, x[:, :24].astype(np.float64))
    gr = ref.backward(pd, cache, z, y[:, :9], m[:, :9])
    lr_ = ref.loss(z, y[:, :9], m[:, :9])
    assert abs(loss - lr_) <= 1e-3 * abs(lr_)
    for k in gr:
        e = _relerr(g[k], gr[k])
        print(f"[mlp-grad {k}] rel err {e:.2e}")
        assert e <= 1e-2, k


def test_adam_steps_track_reference_and_are_deterministic():
    x, y, m = _data(5, 2048)
    p = _params(6)
    runs = []
    for _ in range(2):
        net = resoct.Mlp()
        net.set_weights(p)
        X, Y, M = _dev(x), _dev(y), _dev(m)
        losses = [net.train_step(X, Y, M, 3e-3, want_loss=True) for _ in range(25)]
        runs.append((losses, net.get_weights()))
    assert runs[0][0] == runs[1][0]
    for k in runs[0][1]:
        assert np.array_equal(runs[0][1][k], runs[1][1][k])
    pd = {k: v.astype(np.float64) for k, v in p.items()}
    st = {}
    rl = []
    for _ in range(25):
        z, c = ref.forward(pd, x[:, :24].astype(np.float64))
        rl.append(ref.loss(z, y[:, :9], m[:, :9]))
        pd, st = ref.adam(pd, ref.backward(pd, c, z, y[:, :9], m[:, :9]), st, 3e-3)
    print(f"[mlp-adam] gpu loss {runs[0][0][0]:.4f} -> {runs[0][0][-1]:.4f}, ref {rl[0]:.4f} -> {rl[-1]:.4f}")
    assert runs[0][0][-1] < 0.9 * runs[0][0][0]
    assert abs(runs[0][0][-1] - rl[-1]) <= 0.02 * rl[-1]
