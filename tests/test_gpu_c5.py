"""The 53-qubit, 20-cycle workload: one slice at the full per-slice width,
and the ranking of candidate slicing sets by the runtime models.

* Slice 0 of the width-30 scheme, step by step at its real shapes (stem up
  to 2^30): every step runs on its own from the GPU's input of that step,
  with the autotuner's schedule (as the benchmark runs it), and 2048
  sampled output entries are checked against the oracle's row
  formula on the same input (the local error of each step); the last
  step's 64 values equal the whole plan's slice 0.  FP32 and split FP16,
  bound 1e-5 relative L2 per step.
* Candidate schemes: slicing sets of the chosen order from the randomised
  greedy slicer, and 32 other stem orders (seeded trials of the linear
  stem search, sliced greedily).  The analytic and MLP models predict
  every candidate's total time (per-slice time x 2^|E_s|, paper §A.1; the
  candidates' branches merged up to 12 labels); six
  candidates spread over the analytic ranking
  are measured (slice 0, tuned schedules), both models must order them like
  the measurements (Spearman rank correlation), and the MLP, trained on the
  scheme's own measured steps, must predict the measured times more closely
  than the analytic model.

The full FP64 chain of a 2^30 slice is not run (hours on the host); the
per-step local parity pins every step instead.
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan, planner  # noqa: E402
from paper_2005_06787_amd import _capi as C  # noqa: E402
from paper_2005_06787_amd import runtime_model as rm  # noqa: E402

CFG = configs.C5_53Q_M20
MBR = 12   # merge bound of the ranked candidate plans (the MLP's training shapes)


@pytest.fixture(scope="module")
def scheme():
    circ, oq, closed = configs.circuit_case(CFG)
    pb = planner.CircuitProblem(circ, oq, closed)
    order, sliced, peak, tc = planner.find_scheme(pb.tlabels, CFG["order_trials"],
                                                  CFG["order_seed"], max_width=CFG["max_width"],
                                                  forbid=pb.forbid,
                                                  local_window=CFG["local_window"])
    assert peak <= CFG["max_width"]
    net = planner.scheme_network(pb, order, sliced)
    print(f"53-qubit scheme: {len(sliced)} sliced labels, peak width {peak}, "
          f"log2 tc {np.log2(tc):.1f}, {len(net['branches'])} branches")
    return pb, order, sliced, net


def _fix(labels, data, sliced):
    return stemnet._fix(list(labels), np.asarray(data, np.complex128), {x: 0 for x in sliced})


@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_slice0_full_width_local_error_per_step(scheme, precision, tmp_path):
    _, _, sliced, net = scheme
    cache = str(tmp_path / "tune.txt")
    sl = set(sliced)
    whole = Plan(net, precision=precision)
    ref_final = whole.contract(0, 1).cpu().numpy()[0]
    peak = whole.summary()["peak_rank"]
    whole.close()
    assert CFG["max_width"] - 2 <= peak <= CFG["max_width"]

    rng = np.random.Generator(np.random.PCG64(5005))
    labels = list(net["stem"]["labels"])
    x = torch.from_numpy(np.ascontiguousarray(net["stem"]["data"], np.complex64).reshape(-1)).cuda()
    o_labels, o_stem = _fix(labels, net["stem"]["data"], sl)   # oracle's slice-0 stem
    worst = 0.0
    for i, br in enumerate(net["branches"]):
        blab = list(br["labels"])
        shared = [a for a in labels if a in blab and a not in sl]
        out_labels = [a for a in labels if a not in shared and a not in sl] + \
            [a for a in blab if a not in labels and a not in sl]
        step_sliced = sorted({a for a in labels + blab if a in sl})
        one = {"open_labels": out_labels, "sliced_labels": step_sliced, "proj_labels": [],
               "stem": {"labels": labels}, "branches": [br]}
        plan = Plan(one, precision=precision, stem_device=x)
        plan.tune(slices_in_flight=1, reps=1, cache_path=cache)
        y64 = plan.contract(0, 1)[0]
        plan.close()
        y = y64.to(torch.complex64)
        del y64
        n_out = len(out_labels)
        idx = rng.choice(1 << n_out, size=min(2048, 1 << n_out), replace=False)
        b_labels, b_data = _fix(blab, br["data"], sl)
        if i == 0:
            stem_arr = o_stem.reshape(-1)

            def entries(flat, a=stem_arr):
                return a[np.asarray(flat, dtype=np.int64)]
        else:
            def entries(flat, x=x):
                t = torch.from_numpy(np.asarray(flat, dtype=np.int64).reshape(-1)).cuda()
                return x[t].cpu().numpy().astype(np.complex128).reshape(np.shape(flat))
        ref = stemnet.step_rows(o_labels, entries, b_labels, b_data, out_labels, idx)
        got = y[torch.from_numpy(idx).cuda()].cpu().numpy()
        err = stats.rel_l2(got, ref)
        worst = max(worst, err)
        assert err <= 1e-5, (i, err)
        x, labels, o_labels = y, out_labels, out_labels
    final = x.cpu().numpy().astype(np.complex128)
    # the chain's last tensor is slice 0 over the open labels
    order = [labels.index(a) for a in net["open_labels"]]
    final = final.reshape((2,) * len(labels)).transpose(order).reshape(-1)
    chain_err = stats.rel_l2(final, ref_final)
    print(f"{precision}: {len(net['branches'])} steps, worst local relative L2 {worst:.2e}; "
          f"step chain vs whole plan {chain_err:.2e}")
    assert chain_err <= 1e-5


def test_runtime_models_rank_candidate_slicings(scheme, tmp_path):
    pb, order, sliced, net = scheme
    log = str(tmp_path / "tune.txt")
    sets = planner.candidate_slicings(pb.tlabels, order, CFG["n_candidates"],
                                      CFG["candidate_seed"], max_width=CFG["max_width"],
                                      forbid=pb.forbid)
    assert len(sets) >= 100
    # candidate slicing sets of the chosen order, and candidate stem orders
    others = planner.candidate_orders(pb.tlabels, 32, CFG["candidate_seed"] + 1,
                                      max_width=CFG["max_width"], forbid=pb.forbid)
    cands, shapes, analytic = [], [], []
    for o, c in [(order, c) for c in sets] + others:
        net_c = planner.scheme_network(pb, o, c, with_data=False, max_branch_rank=MBR)
        try:   # schemes the library cannot hold (too many sliced labels on a tensor) drop out
            t = rm.scheme_seconds(net_c, "fp32", 1)["analytic_total_s"]
        except C.StemError:
            continue
        cands.append((o, c))
        shapes.append(net_c)
        analytic.append(t)
    analytic = np.array(analytic)
    assert len(cands) > len(sets)

    # measured step times of the scheme itself train the MLP
    base = Plan(planner.scheme_network(pb, order, sliced, max_branch_rank=MBR))
    base.tune(slices_in_flight=1, reps=1, cache_path=log)
    base.close()
    x, us = rm.read_tune_log(log)
    model = rm.fit(x, us, steps=3000, lr=3e-3, seed=0)
    mlp = np.array([rm.scheme_seconds(n, "fp32", 1, model)["mlp_total_s"] for n in shapes])

    ranked = np.argsort(analytic, kind="stable")
    picks = [int(ranked[int(round(q * (len(ranked) - 1)))]) for q in np.linspace(0, 1, 6)]
    measured = []
    for j in picks:
        plan = Plan(planner.scheme_network(pb, cands[j][0], cands[j][1], max_branch_rank=MBR))
        plan.tune(slices_in_flight=1, reps=1, cache_path=log)
        plan.contract(0, 1)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.contract(0, 1)
        b.record()
        b.synchronize()
        measured.append(a.elapsed_time(b) * 1e-3 * 2.0 ** len(cands[j][1]))
        plan.close()
    measured = np.array(measured)
    rho_an = rm.spearman(analytic[picks], measured)
    rho_mlp = rm.spearman(mlp[picks], measured)
    for j, m in zip(picks, measured):
        print(f"candidate {j}: |E_s| {len(cands[j][1])}, log2 s: analytic {np.log2(analytic[j]):.2f}, "
              f"MLP {np.log2(mlp[j]):.2f}, measured {np.log2(m):.2f}")
    err_an = np.median(np.abs(np.log2(analytic[picks] / measured)))
    err_mlp = np.median(np.abs(np.log2(mlp[picks] / measured)))
    print(f"{len(cands)} candidates; Spearman vs measured: analytic {rho_an:.2f}, MLP {rho_mlp:.2f}; "
          f"median |log2 error|: analytic {err_an:.2f}, MLP {err_mlp:.2f}")
    model.close()
    assert rho_an >= 0.6
    assert rho_mlp >= 0.6
    assert err_mlp < err_an
