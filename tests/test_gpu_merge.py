"""Branch merging (paper §A.3) with the merge points picked by a cost model.

On the 30-qubit, 14-cycle circuit (same order and sliced labels): the
plan whose merge points minimise the roofline step cost, and the plan
whose merge points minimise the MLP's predicted step times, both contract
all 2^10 slices faster than the greedy merge, and all plans give the same
amplitudes.  The MLP is trained on the autotuner's measurements of the
unmerged, greedy and roofline plans, so that the step shapes it compares
(single gates up to merged groups) are all among its training shapes.
"""
import time

import pytest

from oracle import stats
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan, planner  # noqa: E402
from paper_2005_06787_amd import runtime_model as rm  # noqa: E402

CFG = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]


def _measure(net, log):
    plan = Plan(net)
    n = 1 << plan.n_sliced
    g = plan.default_slices_in_flight(n)
    plan.tune(slices_in_flight=g, reps=2, cache_path=log)
    out = plan.contract(0, n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        plan.contract(0, n, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 2
    res = out.cpu().numpy()[0]
    steps = plan.summary()["n_steps"]
    plan.close()
    return dt, res, steps, g


def test_cost_model_merge_points_beat_greedy(tmp_path):
    log = str(tmp_path / "tune.txt")
    circ, oq, closed = configs.circuit_case(CFG)
    pb = planner.CircuitProblem(circ, oq, closed)
    order, sliced, _, _ = planner.find_scheme(pb.tlabels, 64, 0, n_sliced=CFG["n_sliced"],
                                              forbid=pb.forbid)
    greedy = planner.scheme_network(pb, order, sliced, merge="greedy", max_branch_rank=12)
    dp = planner.scheme_network(pb, order, sliced, merge="dp", max_branch_rank=12)
    none = planner.scheme_network(pb, order, sliced, merge="none", max_branch_rank=12)
    t_g, a_g, n_g, g = _measure(greedy, log)
    t_d, a_d, n_d, _ = _measure(dp, log)
    t_n, a_n, n_n, _ = _measure(none, log)
    x, us = rm.read_tune_log(log)
    model = rm.fit(x, us, steps=3000, lr=3e-3, seed=0)
    learned = planner.scheme_network(pb, order, sliced, merge="dp", max_branch_rank=12,
                                     step_cost=rm.mlp_step_cost(model, "fp32", g))
    model.close()
    t_m, a_m, n_m, _ = _measure(learned, log)
    print(f"unmerged {n_n} steps {t_n * 1e3:.1f} ms; greedy {n_g} steps {t_g * 1e3:.1f} ms; "
          f"roofline DP {n_d} steps {t_d * 1e3:.1f} ms; MLP DP {n_m} steps {t_m * 1e3:.1f} ms "
          f"(1024 slices)")
    assert stats.rel_l2(a_n, a_g) <= 1e-5
    assert stats.rel_l2(a_d, a_g) <= 1e-5
    assert stats.rel_l2(a_m, a_g) <= 1e-5
    assert t_d < t_g
    assert t_m < t_g
