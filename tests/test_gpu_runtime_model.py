"""What the learned runtime model gains over the analytic one.

Product-launch times are measured by the autotuner on plans of varied
shape (two precisions, two group sizes); the MLP is trained by the
library's kernels on 80 % of the measured step shapes and must predict the
held-out 20 % with a smaller median relative error than the analytic
roofline model (which knows only the datasheet ceilings).
"""
import numpy as np
import pytest

from workloads.networks import random_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan  # noqa: E402
from paper_2005_06787_amd import runtime_model as rm  # noqa: E402


def collect(log_path):
    rng = np.random.Generator(np.random.PCG64(77))
    for i in range(14):
        r = int(rng.integers(14, 21))
        net = random_stem_network(100 + i, stem_rank=r, n_steps=8, s_range=(1, 7),
                                  f_range=(1, 7), n_sliced=5, n_proj=0, n_open_final=6,
                                  rank_bounds=(r - 4, r + 2))
        for precision in ("fp32", "split_fp16"):
            plan = Plan(net, precision=precision)
            for nz in (4, 32):
                plan.tune(slices_in_flight=nz, reps=2, cache_path=log_path)
            plan.close()
    return rm.read_tune_log(log_path)


def test_mlp_beats_analytic_on_held_out_steps(tmp_path):
    x, us = collect(str(tmp_path / "tune.txt"))
    n = len(us)
    print("measured step shapes:", n)
    assert n >= 100
    perm = np.random.Generator(np.random.PCG64(5)).permutation(n)
    test_idx, train_idx = perm[: n // 5], perm[n // 5:]
    model = rm.fit(x[train_idx], us[train_idx], steps=3000, lr=3e-3, seed=0)
    pred_us = np.exp(model.predict(x[test_idx]))
    analytic_us = 2.0 ** x[test_idx, 11] * 1e6
    actual = us[test_idx]
    err_mlp = np.median(np.abs(pred_us / actual - 1.0))
    err_an = np.median(np.abs(analytic_us / actual - 1.0))
    print(f"median relative error: MLP {err_mlp:.3f}, analytic {err_an:.3f}")
    assert err_mlp < err_an
    assert err_mlp < 0.5
    model.close()
