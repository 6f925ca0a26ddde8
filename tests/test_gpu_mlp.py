"""The learned runtime model's HIP kernels against the FP64 oracle.

With identity feature/target scaling the GPU network computes exactly the
oracle's function (oracle/mlp.py): loss, every parameter gradient (closed-
form back-propagation, itself pinned by finite differences in the oracle's
tests) and the Adam update must agree to FP32 accuracy (relative 1e-4).
"""
import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import runtime_model as rm  # noqa: E402

F, H = 12, 64


def _pack(p):
    return np.concatenate([p[k].reshape(-1) for k in omlp.PARAM_NAMES])


def _data(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((n, F))
    t = x[:, 0] - 0.5 * x[:, 3] * x[:, 5] + 0.1 * rng.standard_normal(n)
    return x, t


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30)


def _fp32_params(p):
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


@pytest.mark.parametrize("n", [1, 37, 300])
def test_loss_and_gradients_match_oracle(n):
    p = _fp32_params(omlp.init_params(F, H, seed=3))
    x, t = _data(n, seed=n)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    m = rm.RuntimeMLP(F, H, init_params=_pack(p))
    loss, grad = m.loss_grad(x, t)
    ref_loss, ref_g = omlp.backward(p, x, t)
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    off = 0
    for k in omlp.PARAM_NAMES:
        size = ref_g[k].size
        g = grad[off:off + size].reshape(ref_g[k].shape)
        assert _rel(g, ref_g[k]) <= 1e-4, k
        off += size
    m.close()


def test_adam_steps_match_oracle():
    p = _fp32_params(omlp.init_params(F, H, seed=4))
    x, t = _data(200, seed=9)
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    m = rm.RuntimeMLP(F, H, init_params=_pack(p))
    m.train(x, t, steps=3, lr=1e-3)
    state = {}
    for _ in range(3):
        _, g = omlp.backward(p, x, t)
        omlp.adam_step(p, g, state, lr=1e-3)
    got = m.params().astype(np.float64)
    ref = _pack(p)
    # Adam moves each parameter by about lr * sign(g) per step, so a
    # gradient component within FP32 rounding of zero may step the other
    # way; all but a handful of parameters must agree to FP32 accuracy
    off = np.abs(got - ref) > 1e-5 + 1e-5 * np.abs(ref)
    assert off.mean() < 0.005, off.sum()
    assert _rel(got, ref) <= 1e-3
    m.close()


def test_training_reduces_loss_and_predict_unscales():
    x, t = _data(2000, seed=1)
    m = rm.RuntimeMLP(F, H, seed=0)
    mean, sd = float(t.mean()), float(t.std())
    m.set_scaling(np.zeros(F), np.ones(F), mean, sd)
    first, _ = m.loss_grad(x, t)
    last = m.train(x, t, steps=800, lr=3e-3)
    assert last < 0.2 * first
    y = m.predict(x[:50])
    # predictions are in target units: close to the targets after training
    assert np.sqrt(np.mean((y - t[:50]) ** 2)) < 0.5 * sd
    m.close()
