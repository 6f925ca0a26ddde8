"""FP64 reference of the runtime-model network (forward, backward, Adam).

The network maps a feature row x to a prediction y:
    h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3
with W1 [F x H], W2 [H x H], W3 [H x 1].  Loss over a batch of B rows with
targets t: L = (1/B) sum_b (y_b - t_b)^2.  Gradients are the closed-form
back-propagation of that composition; relu'(0) is taken as 0.  The update is
Adam (Kingma and Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
theta <- theta - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

Pins (tests/test_oracle_mlp.py): every gradient against central finite
differences; the first Adam step moves each parameter by lr*g/(|g|+eps);
a network with hand-set weights gives hand-computed outputs.
"""

from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init_params(n_features: int, hidden: int, seed: int) -> dict:
    """He-style uniform initialisation, seeded (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def layer(fan_in, fan_out):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=(fan_in, fan_out))

    return {
        "W1": layer(n_features, hidden), "b1": np.zeros(hidden),
        "W2": layer(hidden, hidden), "b2": np.zeros(hidden),
        "W3": layer(hidden, 1), "b3": np.zeros(1),
    }


def forward(params: dict, x: np.ndarray):
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ params["W1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ params["W3"] + params["b3"]
    return y[:, 0], {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss(params: dict, x, t) -> float:
    y, _ = forward(params, x)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2))


def backward(params: dict, x, t):
    """Loss and gradients of every parameter (same shapes as params)."""
    y, c = forward(params, x)
    t = np.asarray(t, dtype=np.float64)
    bsz = y.shape[0]
    dy = (2.0 / bsz) * (y - t)                     # dL/dy
    g = {}
    g["W3"] = c["h2"].T @ dy[:, None]
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] @ params["W3"].T
    dz2 = dh2 * (c["z2"] > 0.0)
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["W2"].T
    dz1 = dh1 * (c["z1"] > 0.0)
    g["W1"] = c["x"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), g


def adam_step(params: dict, grads: dict, state: dict, lr=1e-3, beta1=0.9,
              beta2=0.999, eps=1e-8) -> None:
    """In-place Adam update; ``state`` holds m, v per parameter and step t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in PARAM_NAMES:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1.0 - beta1) * grads[k]
        v[...] = beta2 * v + (1.0 - beta2) * grads[k] ** 2
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
