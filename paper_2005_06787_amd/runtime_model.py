"""Runtime models of stem plans: the analytic roofline model and the learned
MLP (C-ABI stem_cost_analytic, stem_step_features, stem_mlp_*).

Both rank candidate slicing sets / stem orders by predicted contraction
time (paper §A.1: the cost of a scheme is the sum of its steps' costs,
times the number of slices).  The MLP predicts the log time of one product
launch from the step's features; it is trained on the autotuner's measured
step timings, by the library's own HIP kernels.  This module marshals
arguments and reads the autotuner's measurement log.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _capi as C
from .stem import _Desc, _stream_handle

N_FEATURES = C.STEM_N_FEATURES


def plan_steps(net: dict, precision: str = "fp32") -> list:
    """Step infos (ctypes structs) of a network, on the host."""
    # the step shapes depend on the labels only
    d = _Desc(net, precision, shapes_only=True)
    n = ctypes.c_int32()
    C.check(C.lib().stem_plan_steps(ctypes.byref(d.desc), None, 0, ctypes.byref(n)))
    arr = (C.stem_step_info * max(1, n.value))()
    C.check(C.lib().stem_plan_steps(ctypes.byref(d.desc), arr, n.value, ctypes.byref(n)))
    return list(arr)[: n.value]


def step_info_from_shape(log2m: int, log2k: int, log2n: int, amode: int, cmode: int):
    s = C.stem_step_info()
    s.M, s.K, s.N = 1 << log2m, 1 << log2k, 1 << log2n
    s.flops = 8.0 * s.M * s.K * s.N
    s.bytes = 8.0 * (s.M * s.K + s.M * s.N + s.K * s.N)
    s.amode, s.cmode = amode, cmode
    return s


def features(steps, precision: str, slices_in_flight: int) -> np.ndarray:
    """[n_steps, N_FEATURES] float32 features of product launches."""
    out = np.zeros((len(steps), N_FEATURES), dtype=np.float32)
    prec = C.PRECISIONS[precision]
    for i, s in enumerate(steps):
        C.check(C.lib().stem_step_features(ctypes.byref(s), prec, int(slices_in_flight),
                                           out[i].ctypes.data_as(C._f32p_)))
    return out


def analytic_seconds(steps, precision: str, slices_in_flight: int, n_slices: int,
                     hw: dict | None = None) -> float:
    arr = (C.stem_step_info * max(1, len(steps)))(*steps)
    h = None
    if hw is not None:
        h = C.stem_hw(hw["hbm_bytes_per_s"], hw["fp32_flops_per_s"], hw["fp16_flops_per_s"],
                      hw["launch_s"])
    out = ctypes.c_double()
    C.check(C.lib().stem_cost_analytic(arr, len(steps), C.PRECISIONS[precision],
                                       int(slices_in_flight), int(n_slices),
                                       ctypes.byref(h) if h is not None else None,
                                       ctypes.byref(out)))
    return out.value


def read_tune_log(path: str):
    """Measured product launches from the autotuner's log: (features, us).

    Every line is one schedule's time; the model learns the best schedule's
    time per step shape, so only the fastest line of each shape is kept.
    """
    best = {}
    with open(path) as f:
        for line in f:
            p = line.split()
            if not ((len(p) == 13 and p[0] == "stem-tune-v1")
                    or (len(p) == 14 and p[0] == "stem-tune-v2")):
                continue
            prec, am, cm, lm, lk, ln, nz = (int(x) for x in p[1:8])
            us = float(p[-1])
            key = (prec, am, cm, lm, lk, ln, nz)
            if key not in best or us < best[key]:
                best[key] = us
    names = {v: k for k, v in C.PRECISIONS.items()}
    rows, times = [], []
    for (prec, am, cm, lm, lk, ln, nz), us in sorted(best.items()):
        s = step_info_from_shape(lm, lk, ln, am, cm)
        rows.append(features([s], names[prec], nz)[0])
        times.append(us)
    return np.array(rows, dtype=np.float32).reshape(-1, N_FEATURES), np.array(times)


def he_init(n_features: int, hidden: int, seed: int) -> np.ndarray:
    """Seeded He-uniform initial parameters, packed as the C-ABI expects."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def layer(fi, fo):
        lim = math.sqrt(6.0 / fi)
        return rng.uniform(-lim, lim, size=(fi, fo))

    parts = [layer(n_features, hidden), np.zeros(hidden), layer(hidden, hidden), np.zeros(hidden),
             layer(hidden, 1), np.zeros(1)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


class RuntimeMLP:
    """The learned step-time model on the current GPU."""

    def __init__(self, n_features: int = N_FEATURES, hidden: int = 64, init_params=None,
                 seed: int = 0):
        import torch

        self._torch = torch
        self.n_features, self.hidden = n_features, hidden
        self.n_params = int(C.lib().stem_mlp_n_params(n_features, hidden))
        p = he_init(n_features, hidden, seed) if init_params is None else \
            np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        h = ctypes.c_void_p()
        C.check(C.lib().stem_mlp_create(n_features, hidden, p.ctypes.data_as(C._f32p_),
                                        ctypes.byref(h)))
        self._h = h

    def set_scaling(self, x_mean, x_inv_std, t_mean: float, t_std: float):
        xm = np.ascontiguousarray(np.asarray(x_mean, dtype=np.float32))
        xs = np.ascontiguousarray(np.asarray(x_inv_std, dtype=np.float32))
        C.check(C.lib().stem_mlp_set_scaling(self._h, xm.ctypes.data_as(C._f32p_),
                                             xs.ctypes.data_as(C._f32p_), float(t_mean),
                                             float(t_std)))

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        C.check(C.lib().stem_mlp_get_params(self._h, out.ctypes.data_as(C._f32p_)))
        return out

    def _dev(self, a, shape=None):
        t = self._torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")
        return t.reshape(shape) if shape is not None else t

    def loss_grad(self, x, t):
        torch = self._torch
        xd, td = self._dev(x), self._dev(t)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        grad = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        C.check(C.lib().stem_mlp_loss_grad(self._h, ctypes.c_void_p(xd.data_ptr()),
                                           ctypes.c_void_p(td.data_ptr()), len(td),
                                           ctypes.c_void_p(loss.data_ptr()),
                                           ctypes.c_void_p(grad.data_ptr()), _stream_handle(None)))
        return float(loss.item()), grad.cpu().numpy()

    def train(self, x, t, steps: int, lr: float = 1e-3) -> float:
        torch = self._torch
        xd, td = self._dev(x), self._dev(t)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        C.check(C.lib().stem_mlp_train(self._h, ctypes.c_void_p(xd.data_ptr()),
                                       ctypes.c_void_p(td.data_ptr()), len(td), int(steps),
                                       float(lr), ctypes.c_void_p(loss.data_ptr()),
                                       _stream_handle(None)))
        return float(loss.item())

    def predict(self, x) -> np.ndarray:
        torch = self._torch
        xd = self._dev(x)
        n = xd.shape[0]
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        C.check(C.lib().stem_mlp_predict(self._h, ctypes.c_void_p(xd.data_ptr()), n,
                                         ctypes.c_void_p(y.data_ptr()), _stream_handle(None)))
        return y.cpu().numpy()

    def close(self):
        if getattr(self, "_h", None):
            C.lib().stem_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(x: np.ndarray, us: np.ndarray, hidden: int = 64, steps: int = 3000, lr: float = 3e-3,
        seed: int = 0) -> RuntimeMLP:
    """Train a RuntimeMLP on (features, measured microseconds)."""
    t = np.log(np.asarray(us, dtype=np.float64))
    xm = x.mean(axis=0)
    xsd = x.std(axis=0)
    inv = np.where(xsd > 1e-6, 1.0 / np.maximum(xsd, 1e-6), 1.0)
    m = RuntimeMLP(x.shape[1], hidden, seed=seed)
    m.set_scaling(xm, inv, float(t.mean()), float(max(t.std(), 1e-3)))
    m.train(x, t.astype(np.float32), steps, lr)
    return m


def scheme_seconds(net: dict, precision: str = "fp32", slices_in_flight: int = 1,
                   model: "RuntimeMLP | None" = None) -> dict:
    """Predicted contraction time of a scheme's network (labels suffice).

    Returns seconds per slice and for all 2^|E_s| slices (§A.1: the cost of a
    sliced scheme is the per-slice cost times the number of slices), from
    the analytic model and, when ``model`` is given, from the MLP: its
    product-launch times (a launch carries ``slices_in_flight`` slices) plus
    the analytic cost of the permutes and the final accumulation.
    """
    steps = plan_steps(net, precision)
    n_slices = 2.0 ** len(net["sliced_labels"])
    g = max(1, int(slices_in_flight))
    per_group = analytic_seconds(steps, precision, g, g)
    out = {"analytic_slice_s": per_group / g, "analytic_total_s": per_group / g * n_slices}
    if model is not None:
        # analytic cost of everything but the product launches
        bare = []
        for s in steps:
            c = C.stem_step_info()
            ctypes.memmove(ctypes.byref(c), ctypes.byref(s), ctypes.sizeof(c))
            c.permuted = 0
            bare.append(c)
        launch = analytic_seconds([], precision, g, g)
        rest = per_group - (analytic_seconds(bare, precision, g, g) - launch)
        pred_us = np.exp(model.predict(features(steps, precision, g))) if steps else np.zeros(0)
        mlp_group = float(pred_us.sum()) * 1e-6 + rest
        out["mlp_slice_s"] = mlp_group / g
        out["mlp_total_s"] = mlp_group / g * n_slices
    return out


def spearman(a, b) -> float:
    """Spearman rank correlation of two sequences (average ranks for ties)."""
    def ranks(x):
        x = np.asarray(x, dtype=np.float64)
        order = np.argsort(x, kind="stable")
        r = np.empty(len(x))
        i = 0
        while i < len(x):
            j = i
            while j + 1 < len(x) and x[order[j + 1]] == x[order[i]]:
                j += 1
            r[order[i:j + 1]] = 0.5 * (i + j)
            i = j + 1
        return r
    ra, rb = ranks(a), ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = math.sqrt(float((ra * ra).sum() * (rb * rb).sum()))
    return float((ra * rb).sum() / den) if den > 0 else 0.0


def mlp_step_cost(model: "RuntimeMLP", precision: str = "fp32", slices_in_flight: int = 128):
    """step_cost(r_in, s, f) for the planner's branch merging from the MLP:
    the predicted time of one product launch of that shape (stem read
    M-fast, output in block order), per slice.  Predictions are cached."""
    cache = {}
    g = max(1, int(slices_in_flight))

    def cost(r_in, s, f):
        key = (r_in, s, f)
        if key not in cache:
            st = step_info_from_shape(r_in - s, s, f, 1, 1 if r_in - s >= 4 else 0)
            us = float(np.exp(model.predict(features([st], precision, g))[0]))
            cache[key] = us * 1e-6 / g
        return cache[key]
    return cost
