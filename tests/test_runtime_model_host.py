"""Host-side parts of the runtime models (no GPU): step shapes of a
descriptor, the analytic roofline model (paper §A.1 step cost) against its
closed form, the step features, and the autotuner-log reader."""
import math

import numpy as np
import pytest

from paper_2005_06787_amd import runtime_model as rm
from paper_2005_06787_amd import stem_plan_validate
from workloads.networks import random_stem_network

HW = {"hbm_bytes_per_s": 8e12, "fp32_flops_per_s": 157.3e12, "fp16_flops_per_s": 2.5e15,
      "launch_s": 4e-6}


@pytest.mark.parametrize("seed", range(5))
def test_plan_steps_match_summary(seed):
    net = random_stem_network(seed, stem_rank=12, n_steps=8, s_range=(1, 5), f_range=(1, 5),
                              n_open_final=5, rank_bounds=(1, 15))
    steps = rm.plan_steps(net)
    summ = stem_plan_validate(net)
    assert len(steps) == summ["n_steps"]
    assert sum(s.permuted for s in steps) == summ["n_permutes"]
    assert sum(s.flops for s in steps) == summ["flops_per_slice"]
    for s in steps:
        assert s.M * s.K == 2 ** s.rank_in
        assert s.M * s.N == 2 ** s.rank_out
        assert s.amode in (0, 1) and s.cmode in (0, 1)


@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_analytic_model_closed_form(precision):
    net = random_stem_network(3, stem_rank=14, n_steps=6, s_range=(2, 6), f_range=(2, 6),
                              n_sliced=4, n_open_final=6, rank_bounds=(1, 16))
    steps = rm.plan_steps(net, precision)
    g, n_slices = 5, 16
    rate = HW["fp32_flops_per_s"] if precision == "fp32" else HW["fp16_flops_per_s"] / 3
    per_group = HW["launch_s"]
    for s in steps:
        m, k, n = s.M, s.K, s.N
        t = max(g * 8 * (m * k + m * n + k * n) / HW["hbm_bytes_per_s"], g * 8 * m * k * n / rate)
        per_group += t + HW["launch_s"]
        if s.permuted:
            per_group += g * 16 * 2 ** s.rank_in / HW["hbm_bytes_per_s"] + HW["launch_s"]
    want = math.ceil(n_slices / g) * per_group
    got = rm.analytic_seconds(steps, precision, g, n_slices, HW)
    assert got == pytest.approx(want, rel=1e-12)
    # the default hardware description is the same one
    assert rm.analytic_seconds(steps, precision, g, n_slices) == pytest.approx(got, rel=1e-12)


def test_features():
    s = rm.step_info_from_shape(20, 5, 3, 1, 1)
    f = rm.features([s], "split_fp16", 64)[0]
    assert list(f[:9]) == [20, 5, 3, 6, 1, 1, 0, 1, 0]
    nbytes = 64 * 8 * (2 ** 25 + 2 ** 23 + 2 ** 8)
    assert f[9] == pytest.approx(math.log2(nbytes), rel=1e-6)
    assert f[10] == pytest.approx(math.log2(64 * 8 * 2 ** 28), rel=1e-6)
    t = max(nbytes / 8e12, 64 * 8 * 2 ** 28 / (2.5e15 / 3)) + 4e-6
    assert f[11] == pytest.approx(math.log2(t), rel=1e-6)


def test_read_tune_log(tmp_path):
    p = tmp_path / "log.txt"
    p.write_text("stem-tune-v1 0 1 1 20 5 5 64 2 4 4096 -1 120.5\n"
                 "stem-tune-v1 0 1 1 20 5 5 64 1 4 4096 -1 100.0\n"
                 "garbage line\n"
                 "stem-tune-v1 1 0 1 18 3 4 8 4 1 1024 0 7.25\n"
                 "stem-tune-v2 0 1 1 20 5 5 64 1 2 4096 -1 1 90.0\n"
                 "stem-tune-v2 0 1 1 16 3 4 64 1 2 4096 -1 0 3.5\n")
    x, us = rm.read_tune_log(str(p))
    assert x.shape == (3, rm.N_FEATURES)
    assert sorted(us.tolist()) == [3.5, 7.25, 90.0]


def test_he_init_shapes():
    p = rm.he_init(12, 64, 0)
    assert p.size == 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    assert np.all(np.abs(p[:12 * 64]) <= math.sqrt(6 / 12))
