"""Isolated stem chains (random complex Gaussian branches, counter-based
initial stem) in the three precisions against the FP64 oracle.

* 2^22 stem, 16 steps: the whole chain against the oracle's FP64 chain.
* 2^30 stem, 40 steps (the real per-slice shape): every step run on its own
  from the GPU's FP32 input of that step, with the autotuner's schedule
  (as the benchmark runs it: for FP32 mostly the 3M product), and 4096
  sampled output entries checked against the oracle's row formula on that
  same input (the local error of each step).

Bounds: FP32 and split FP16 relative L2 <= 1e-5; split BF16 5e-4 (8 + 8
significant bits per factor).
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads import tensors as wt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan, stem_fill_counter  # noqa: E402

TOL = {"fp32": 1e-5, "split_fp16": 1e-5, "split_bf16": 5e-4}


def _net(iso, branches=None):
    return {"open_labels": iso["final_labels"], "sliced_labels": [], "proj_labels": [],
            "stem": {"labels": iso["stem_labels"]},
            "branches": iso["branches"] if branches is None else branches}


def _device_stem(iso):
    r = len(iso["stem_labels"])
    x = torch.empty(1 << r, dtype=torch.complex64, device="cuda")
    stem_fill_counter(x, iso["stem_seed"], iso["stem_scale_log2"])
    return x


@pytest.mark.parametrize("precision", ["fp32", "split_fp16", "split_bf16"])
def test_chain_2e22_against_fp64_chain(precision):
    iso = wt.random_isolated_stem(22, 16, seed=33)
    x = _device_stem(iso)
    plan = Plan(_net(iso), precision=precision, stem_device=x)
    got = plan.contract().cpu().numpy()[0]
    plan.close()
    r = len(iso["stem_labels"])
    stem = wt.counter_stem_entries(iso["stem_seed"], np.arange(1 << r),
                                   iso["stem_scale_log2"]).reshape((2,) * r)
    onet = _net(iso, [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                      for b in iso["branches"]])
    onet["stem"] = {"labels": iso["stem_labels"], "data": stem}
    ref, _ = stemnet.run_slice(onet, 0, 0)
    err = stats.rel_l2(got, ref.reshape(-1))
    print(f"{precision}: 2^22 chain of 16 steps, relative L2 {err:.2e}")
    assert err <= TOL[precision] * 4  # 16 steps of local error


@pytest.mark.parametrize("precision", ["fp32", "split_fp16", "split_bf16"])
def test_full_size_local_error_per_step(precision, tmp_path):
    iso = wt.random_isolated_stem(30, 40, seed=3)
    cache = str(tmp_path / "tune.txt")
    x = _device_stem(iso)
    labels = list(iso["stem_labels"])
    rng = np.random.Generator(np.random.PCG64(3003))
    n_steps = len(iso["branches"]) if precision != "split_bf16" else 8
    worst = 0.0
    for i, br in enumerate(iso["branches"][:n_steps]):
        shared = [a for a in labels if a in br["labels"]]
        out_labels = [a for a in labels if a not in shared] + \
            [a for a in br["labels"] if a not in labels]
        net = {"open_labels": out_labels, "sliced_labels": [], "proj_labels": [],
               "stem": {"labels": labels}, "branches": [br]}
        plan = Plan(net, precision=precision, stem_device=x)
        plan.tune(slices_in_flight=1, reps=1, cache_path=cache)
        y64 = plan.contract()[0]
        plan.close()
        y = y64.to(torch.complex64)
        del y64
        idx = rng.choice(1 << len(out_labels), size=4096, replace=False)

        def entries(flat, x=x):
            t = torch.from_numpy(np.asarray(flat, dtype=np.int64).reshape(-1)).cuda()
            return x[t].cpu().numpy().astype(np.complex128).reshape(np.shape(flat))

        ref = stemnet.step_rows(labels, entries, br["labels"],
                                np.asarray(br["data"], np.complex128), out_labels, idx)
        got = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        err = stats.rel_l2(got, ref)
        worst = max(worst, err)
        assert err <= TOL[precision], (i, err)
        x, labels = y, out_labels
    print(f"{precision}: worst local relative L2 over {n_steps} steps at 2^30: {worst:.2e}")
