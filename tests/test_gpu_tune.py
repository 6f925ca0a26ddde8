"""The launch-schedule autotuner (C-ABI stem_tune).

A schedule's row blocks, column tiles, workgroups and LDS use change only
how the work is spread, never the order in which a product sums, so results
after tuning must be bit-identical to the same arithmetic under any other
such schedule (and to the defaults when no step chose the FP32 3M
product); the cache file must hold one well-formed line per measurement
and be reused without measuring again.
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads.networks import random_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan  # noqa: E402


def _c128(net):
    out = dict(net)
    out["stem"] = {"labels": net["stem"]["labels"],
                   "data": np.asarray(net["stem"]["data"], np.complex128)}
    out["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                       for b in net["branches"]]
    return out


@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_tune_keeps_results_and_caches(tmp_path, precision):
    net = random_stem_network(21, stem_rank=16, n_steps=8, s_range=(2, 6), f_range=(2, 6),
                              n_sliced=3, n_proj=1, n_open_final=6, rank_bounds=(1, 18))
    plan = Plan(net, precision=precision)
    n = 1 << plan.n_sliced
    before = plan.contract(0, n, proj=[0, 1], slices_in_flight=n).clone()
    cache = tmp_path / "tune.txt"
    steps = plan.tune(slices_in_flight=n, reps=2, cache_path=str(cache))
    lines = cache.read_text().split("\n")
    lines = [x for x in lines if x]
    assert len(lines) >= len(steps)
    for line in lines:
        f = line.split()
        assert f[0] == "stem-tune-v2" and len(f) == 14
        assert f[12] in ("0", "1") and (precision == "fp32" or f[12] == "0")
        assert float(f[-1]) > 0
    for s in steps:
        assert s["sched_tm"] in (1, 2, 4) and s["sched_ntw"] in (1, 2, 4, 8)
        assert s["tuned_us"] > 0 and s["tuned_slices"] == n
    after = plan.contract(0, n, proj=[0, 1], slices_in_flight=n)
    if all(s["sched_algo"] == 0 for s in steps):
        assert torch.equal(before, after)
    # the same arithmetic per step under another spread of the work
    plan3 = Plan(net, precision=precision)
    for i, s in enumerate(steps):
        plan3.set_schedule(i, 1, 1, 1024, 0, s["sched_algo"])
    assert torch.equal(plan3.contract(0, n, proj=[0, 1], slices_in_flight=n), after)
    plan3.close()
    onet = _c128(net)
    for p in (0, 1):
        ref = stemnet.sliced_sum(onet, proj=p).reshape(-1)
        assert stats.rel_l2(after[p].cpu().numpy(), ref) <= 1e-5
    # a second plan with the same shapes takes the cached schedules
    plan2 = Plan(net, precision=precision)
    steps2 = plan2.tune(slices_in_flight=n, reps=2, cache_path=str(cache))
    assert len([x for x in cache.read_text().split("\n") if x]) == len(lines)
    for a, b in zip(steps, steps2):
        assert (a["sched_tm"], a["sched_ntw"], a["sched_blocks"], a["sched_lds"],
                a["sched_algo"]) == \
            (b["sched_tm"], b["sched_ntw"], b["sched_blocks"], b["sched_lds"], b["sched_algo"])
    plan.close()
    plan2.close()
