"""Workgroup shape does not change the arithmetic.

A product's 8-wave workgroups (two waves per SIMD sharing one LDS copy of
the branch fragments) spread the same per-row sums over more waves, so
every step run that way gives the same bits as with 4-wave workgroups and
the same tiles, in split FP16, split BF16 and the FP32 3M product; and the
results match the FP64 oracle (relative L2 1e-5; 5e-4 for split BF16,
whose two BF16 terms carry 16 significant bits).
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads.networks import random_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan  # noqa: E402

TOL = {"fp32": 1e-5, "split_fp16": 1e-5, "split_bf16": 5e-4}


def _net(seed):
    return random_stem_network(seed, stem_rank=16, n_steps=6, s_range=(3, 6), f_range=(4, 6),
                               n_sliced=2, n_proj=1, n_open_final=6, rank_bounds=(9, 18))


def _c128(net):
    out = dict(net)
    out["stem"] = {"labels": net["stem"]["labels"],
                   "data": np.asarray(net["stem"]["data"], dtype=np.complex128)}
    out["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                       for b in net["branches"]]
    return out


@pytest.mark.parametrize("seed", [71, 72])
@pytest.mark.parametrize("precision,algo", [("split_fp16", 0), ("split_bf16", 0), ("fp32", 1)])
def test_eight_wave_workgroups_give_the_same_bits(seed, precision, algo):
    net = _net(seed)
    plan = Plan(net, precision=precision)
    steps = plan.steps()
    use = [i for i, s in enumerate(steps)
           if s["cmode"] == 1 and s["M"] % 256 == 0
           and (algo == 0 or (s["K"] % 8 == 0 and s["N"] % 16 == 0))]
    assert use, "no step with whole 8-wave row blocks"
    print(f"network seed {seed} {precision}: steps {use}", flush=True)
    n = 1 << plan.n_sliced
    outs = []
    for lds in ((1, 2, 3) if algo == 1 else (1, 2)):
        for i in use:
            info = plan.set_schedule(i, 2, 2, 4096, lds, algo)
            assert info["sched_lds"] == lds
        outs.append(plan.contract(0, n, proj=[0, 1]).clone())
    for o in outs[1:]:
        assert torch.equal(outs[0], o)
    onet = _c128(net)
    got = outs[-1].cpu().numpy()
    for p in (0, 1):
        ref = stemnet.sliced_sum(onet, proj=p).reshape(-1)
        assert stats.rel_l2(got[p], ref) <= TOL[precision], p
    plan.close()
