"""Batch labels (hyperedges, paper §A.1): a step keeps labels it shares
with the stem when a later branch or the result still carries them, and
runs a batched product, one per assignment of those labels, each with its
own branch sub-matrix.

Random hyperedge networks through the C-ABI against the FP64 oracle (which
keeps such labels as common indices), per slice and projected assignment,
FP32 and split FP16 at relative L2 <= 1e-5; tuned schedules give the same
results; a group of slices per launch is bit-identical to one slice per
launch.
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads.networks import random_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan  # noqa: E402

NETS = [
    # (seed, stem_rank, n_steps, s_range, f_range, n_sliced, n_proj, n_open_final, batch_prob)
    (21, 10, 8, (1, 5), (0, 4), 2, 1, 6, 0.4),
    (22, 14, 8, (2, 6), (2, 6), 2, 1, 8, 0.5),
    (23, 16, 6, (4, 7), (4, 7), 1, 0, 10, 0.5),   # K, N up to 128 per batch index
    (24, 9, 10, (1, 3), (0, 3), 3, 2, 4, 0.6),
    (25, 12, 8, (1, 4), (1, 4), 2, 1, 0, 0.5),    # scalar result
]


def _net(cfg):
    seed, r, n, sr, fr, nsl, npr, nof, bp = cfg
    return random_stem_network(seed, stem_rank=r, n_steps=n, s_range=sr, f_range=fr,
                               n_sliced=nsl, n_proj=npr, n_open_final=nof, batch_prob=bp,
                               rank_bounds=(1, r + 3))


def _c128(net):
    out = dict(net)
    out["stem"] = {"labels": net["stem"]["labels"],
                   "data": np.asarray(net["stem"]["data"], dtype=np.complex128)}
    out["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                       for b in net["branches"]]
    return out


@pytest.mark.parametrize("cfg", NETS, ids=lambda c: f"seed{c[0]}")
@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_batched_steps_match_oracle(cfg, precision):
    net = _net(cfg)
    onet = _c128(net)
    print(f"network seed {cfg[0]} precision {precision}", flush=True)
    plan = Plan(net, precision=precision)
    batched = [s["n_batch"] for s in plan.steps()]
    assert max(batched) > 0, "no batched step drawn"
    n_sl, n_pr = len(net["sliced_labels"]), len(net["proj_labels"])
    projs = list(range(1 << n_pr))
    for s in range(1 << n_sl):
        got = plan.contract(s, s + 1, proj=projs).cpu().numpy()
        for p in projs:
            ref, _ = stemnet.run_slice(onet, s, p)
            err = stats.rel_l2(got[p], ref.reshape(-1))
            assert err <= 1e-5, (s, p, err)
    plan.close()


@pytest.mark.parametrize("cfg", NETS[:3], ids=lambda c: f"seed{c[0]}")
def test_batched_groups_and_tuning(cfg, tmp_path):
    net = _net(cfg)
    plan = Plan(net)
    n = 1 << plan.n_sliced
    one = torch.cat([plan.contract(0, n, slices_in_flight=1)])
    many = plan.contract(0, n, slices_in_flight=n)
    assert torch.equal(one, many)
    plan.tune(slices_in_flight=n, reps=1, cache_path=str(tmp_path / "tune.txt"))
    tuned = plan.contract(0, n, slices_in_flight=n).cpu().numpy()
    plan.close()
    ref = stemnet.sliced_sum(_c128(net)).reshape(-1)
    assert stats.rel_l2(tuned[0], ref) <= 1e-5
