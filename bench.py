"""Benchmark of the sliced stem contraction on one MI355X.

Workload (default): the 5x6-grid, 14-cycle random circuit (30 qubits) with
6 open qubits (a 64-amplitude batch) and 10 sliced labels, i.e. 2^10
slices; one *step* is one pass of the whole hot path over that batch --
every slice contracted (stem permutes + complex products on the matrix
cores) and summed in FP64 into the 64 amplitudes.  The plan is made before
the timed region (preprocessing is not timed, as in the paper).

Prints one JSON line: TFLOP/s (8 real flops per complex multiply-add,
summed over the steps' useful products) and slices/s for the FP32 path,
the same for the split-FP16 path, the amplitude error of both against the
FP64 oracle on sampled slices, a roofline entry for the dominant kernel
(the FP32 product, HBM-bound) and the oracle's own rate on the host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_PEAK_FLOPS = 157.3e12   # MI355X dense FP32 (MFMA)
HBM_PEAK_GBS = 8000.0
# HBM traffic of the FP32 product kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs (scaled by a 1 GiB copy), recorded with a hash of the
# kernel's sources; reported only while the sources still match.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cgemm_f32_c2_5x6_m14_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_06787_amd", "csrc", f)
                  for f in ("gemm_f32.hip", "device_common.h")]


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(bytes_per_launch: float):
    """HBM bytes per product launch measured by the counters, when the
    record is of these kernel sources and of launches of this size."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    if abs(rec.get("algorithmic_bytes_per_launch", 0) - bytes_per_launch) > 1e-6 * bytes_per_launch:
        return None
    return rec.get("bytes_per_launch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_net():
    from paper_2005_06787_amd import planner
    from workloads import configs, tensors
    from workloads.circuits import make_circuit

    cfg = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]
    circ = make_circuit(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"])
    oq = configs.open_qubits(cfg)
    pre = tensors.split_open_prefix(circ["n_qubits"], oq, cfg["prefix_seed"])
    closed = dict(zip(pre["closed"], pre["closed_bits"]))
    net = planner.plan_circuit(circ, oq, closed, n_sliced=cfg["n_sliced"], trials=64, seed=0,
                               max_branch_rank=cfg["max_branch_rank"])
    return net, cfg


def batched_workload(steps: int, tune_cache=None):
    """8 seeded 40-qubit circuits (5x8 grid, 10-14 cycles, sliced to widths
    20-24), the first 512 slices of each, as one graph launch."""
    import torch

    from paper_2005_06787_amd import Batch, Plan, ceilings, planner
    from workloads import configs, tensors
    from workloads.circuits import block_qubits, make_circuit

    cfg = configs.BATCH_5X8
    plans, ranges, flops, nbytes, ws_max = [], [], 0.0, 0.0, 0
    t0 = time.perf_counter()
    for j, (cyc, w) in enumerate(zip(cfg["cycles"], cfg["widths"])):
        circ = make_circuit(cfg["rows"], cfg["cols"], cyc, cfg["circuit_seed0"] + j)
        oq = block_qubits(cfg["rows"], cfg["cols"], cfg["open_rows"], cfg["open_cols"])
        pre = tensors.split_open_prefix(circ["n_qubits"], oq, cfg["prefix_seed0"] + j)
        closed = dict(zip(pre["closed"], pre["closed_bits"]))
        net = planner.plan_circuit(circ, oq, closed, max_width=w, trials=8, seed=j)
        plan = Plan(net)
        n = min(cfg["slices_each"], 1 << plan.n_sliced)
        group = min(n, max(1, (8 << 30) // plan.workspace_bytes(1)))
        plan.tune(slices_in_flight=group, reps=2, cache_path=tune_cache)
        plans.append(plan)
        ranges.append((0, n))
        flops += plan.summary()["flops_per_slice"] * n
        nbytes += plan.summary()["bytes_per_slice"] * n
        ws_max = max(ws_max, plan.workspace_bytes(group))
        log(f"batched circuit {j}: {cyc} cycles, width {net['stats']['peak_width']}, "
            f"{len(net['sliced_labels'])} sliced labels, group {group}")
    log(f"batched workload planned and tuned in {time.perf_counter() - t0:.1f} s")
    ws_bytes = len(plans) * max(p.workspace_bytes(min(r[1], max(1, (8 << 30) // p.workspace_bytes(1))))
                                for p, r in zip(plans, ranges))
    batch = Batch(plans, ranges, ws_bytes=ws_bytes)
    batch.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.launch()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    n_sl = sum(r[1] - r[0] for r in ranges)
    out = {"workload": "8 circuits, 5x8 grid (40 qubits), 10-14 cycles, widths 20-24, "
                       "first 512 slices each, one graph launch, FP32",
           "slices": n_sl, "ms_per_launch": round(dt * 1e3, 3),
           "slices_per_s": round(n_sl / dt, 1), "tflops": round(flops / dt / 1e12, 3),
           "algorithmic_gbs": round(nbytes / dt / 1e9, 1)}
    batch.close()
    for p in plans:
        p.close()
    torch.cuda.empty_cache()
    # both copy ceilings: the stems of these circuits (2^20-2^24 entries) fit the
    # 256 MiB last-level cache one at a time, but a plan's group of slices in
    # flight does not (its workspace is the working set of one step)
    hbm = ceilings.copy_gbs(4 << 30, 16)
    llc = ceilings.copy_gbs(64 << 20, 16, reps=50)
    out.update({"largest_group_workspace_gib": round(ws_max / 2**30, 2),
                "hbm_copy_gbs": round(hbm, 1), "llc_copy_gbs_64mib": round(llc, 1),
                "frac_of_hbm_copy": round(nbytes / dt / 1e9 / hbm, 3),
                "frac_of_llc_copy": round(nbytes / dt / 1e9 / llc, 3)})
    return out


def isolated_stem(steps: int, tune_cache=None):
    """The isolated stem at its real shape: a 2^30 complex64 stem (8 GiB),
    40 steps with random complex Gaussian branches, in the three precisions."""
    import torch

    from paper_2005_06787_amd import Plan, stem_fill_counter
    from workloads import configs
    from workloads import tensors as wt

    c = configs.ISOLATED_STEM
    iso = wt.random_isolated_stem(c["n_rank"], c["n_steps"], seed=c["seed"])
    x = torch.empty(1 << c["n_rank"], dtype=torch.complex64, device="cuda")
    stem_fill_counter(x, iso["stem_seed"], iso["stem_scale_log2"])
    net = {"open_labels": iso["final_labels"], "sliced_labels": [], "proj_labels": [],
           "stem": {"labels": iso["stem_labels"]}, "branches": iso["branches"]}
    out = {"workload": "isolated stem, 2^30 complex64, 40 steps, branches of rank 6-14 "
                       "sharing 4-8 labels"}
    for precision in ("fp32", "split_fp16", "split_bf16"):
        plan = Plan(net, precision=precision, stem_device=x)
        summ = plan.summary()
        plan.tune(slices_in_flight=1, reps=2, cache_path=tune_cache)
        res = plan.contract()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.contract(out=res)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[precision] = {"ms_per_chain": round(dt * 1e3, 3),
                          "tflops": round(summ["flops_per_slice"] / dt / 1e12, 2),
                          "algorithmic_gbs": round(summ["bytes_per_slice"] / dt / 1e9, 1)}
        log(f"isolated stem {precision}: {dt * 1e3:.1f} ms, "
            f"{summ['flops_per_slice'] / dt / 1e12:.1f} TFLOP/s")
        del res
        plan.close()
    out["flops_per_chain"] = summ["flops_per_slice"]
    out["bytes_per_chain"] = summ["bytes_per_slice"]
    del x
    torch.cuda.empty_cache()
    return out


def slice_53q(steps: int, tune_cache=None):
    """One slice of the 53-qubit, 20-cycle circuit at its full per-slice
    width (stem up to 2^30): slice 0 of the width-30 scheme, FP32 against
    split FP16."""
    import torch

    from paper_2005_06787_amd import Plan, planner
    from workloads import configs

    cfg = configs.C5_53Q_M20
    t0 = time.perf_counter()
    circ, oq, closed = configs.circuit_case(cfg)
    pb = planner.CircuitProblem(circ, oq, closed)
    order, sliced, peak, tc = planner.find_scheme(pb.tlabels, cfg["order_trials"],
                                                  cfg["order_seed"], max_width=cfg["max_width"],
                                                  forbid=pb.forbid,
                                                  local_window=cfg["local_window"])
    net = planner.scheme_network(pb, order, sliced)
    log(f"53-qubit scheme planned in {time.perf_counter() - t0:.1f} s: {len(sliced)} sliced "
        f"labels, peak width {peak}, {len(net['branches'])} steps")
    out = {"workload": f"53 qubits (6x9 grid less one site), 20 cycles, slice 0 of a width-"
                       f"{peak} scheme with {len(sliced)} sliced labels, {len(net['branches'])} "
                       f"steps"}
    for precision in ("fp32", "split_fp16"):
        plan = Plan(net, precision=precision)
        summ = plan.summary()
        plan.tune(slices_in_flight=1, reps=1, cache_path=tune_cache)
        res = plan.contract(0, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.contract(0, 1, out=res)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[precision] = {"ms_per_slice": round(dt * 1e3, 3),
                          "tflops": round(summ["flops_per_slice"] / dt / 1e12, 2),
                          "algorithmic_gbs": round(summ["bytes_per_slice"] / dt / 1e9, 1)}
        log(f"53-qubit slice {precision}: {dt * 1e3:.1f} ms, "
            f"{summ['flops_per_slice'] / dt / 1e12:.1f} TFLOP/s")
        del res
        plan.close()
    out["flops_per_slice"] = summ["flops_per_slice"]
    out["bytes_per_slice"] = summ["bytes_per_slice"]
    torch.cuda.empty_cache()
    return out


def locally_optimised_30q(steps: int, tune_cache=None):
    """The headline circuit and slice count with the planner's stem-focused
    local optimisation (windows of 5 tensors re-ordered after every slicing
    pick): a smaller stem and fewer flops per slice for the same amplitudes."""
    import torch

    from paper_2005_06787_amd import Plan, planner
    from workloads import configs

    cfg = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]
    circ, oq, closed = configs.circuit_case(cfg)
    net = planner.plan_circuit(circ, oq, closed, n_sliced=cfg["n_sliced"], trials=64, seed=0,
                               local_window=5, max_branch_rank=cfg["max_branch_rank"])
    out = {"workload": "5x6 grid, 14 cycles, 30 qubits, 2^10 slices, plan with local "
                       "optimisation (window 5)"}
    for precision in ("fp32", "split_fp16"):
        plan = Plan(net, precision=precision)
        summ = plan.summary()
        n = int(summ["n_slices"])
        plan.tune(slices_in_flight=plan.default_slices_in_flight(n), reps=2, cache_path=tune_cache)
        res = plan.contract(0, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.contract(0, n, out=res)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[precision] = {"ms_per_step": round(dt * 1e3, 3), "slices_per_s": round(n / dt, 1),
                          "tflops": round(summ["flops_per_slice"] * n / dt / 1e12, 2)}
        log(f"locally optimised 30-qubit plan {precision}: {n / dt:.0f} slices/s")
        plan.close()
    out.update({"peak_rank": summ["peak_rank"], "n_steps": summ["n_steps"],
                "flops_per_slice": summ["flops_per_slice"],
                "bytes_per_slice": summ["bytes_per_slice"]})
    return out


def two_sided_30q(steps: int, tune_cache=None):
    """The headline circuit's scheme (same order and sliced labels) as two
    stems meeting at the root: the left stem grows from the start of the
    order, the right stem from its end, and the join contracts them over
    the cut.  Two cuts: the one with the smallest modelled time (roofline
    of both sides' products plus the join) and the earliest one modelled
    within 5 % of it (a long shared index); all 2^10 slices, FP32."""
    import torch

    from paper_2005_06787_amd import Join, Plan, planner
    from paper_2005_06787_amd.stem import stem_plan_validate
    from workloads import configs

    cfg = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]
    circ, oq, closed = configs.circuit_case(cfg)
    pb = planner.CircuitProblem(circ, oq, closed)
    order, sliced, _, _ = planner.find_scheme(pb.tlabels, 64, 0, n_sliced=cfg["n_sliced"],
                                              forbid=pb.forbid)
    mbr = cfg["max_branch_rank"]
    cand = []
    for h in range(len(order) // 2, len(order) - 1):
        try:
            left, right, _ = planner.two_sided_networks(pb, order, sliced, h, with_data=False,
                                                        max_branch_rank=mbr)
            sl, sr = stem_plan_validate(left), stem_plan_validate(right)
        except Exception:   # a side above the rank limits
            continue
        k = len(set(left["open_labels"]) & set(right["open_labels"]))
        a, b = len(left["open_labels"]) - k, len(right["open_labels"]) - k
        by = sl["bytes_per_slice"] + sr["bytes_per_slice"] + 8.0 * 2 ** k * (2 ** a + 2 ** b)
        fl = sl["flops_per_slice"] + sr["flops_per_slice"] + 8.0 * 2 ** (k + a + b)
        cand.append((max(by / 5e12, fl / 1.2e14), h, fl))
    t_best = min(c[0] for c in cand)
    best = min(cand)
    deep = min((c for c in cand if c[0] <= 1.05 * t_best), key=lambda c: c[1])
    one = planner.scheme_network(pb, order, sliced, max_branch_rank=mbr)
    p1 = Plan(one)
    n = 1 << p1.n_sliced
    ref = p1.contract(0, n).cpu().numpy()[0]
    p1.close()
    out = {"workload": "5x6 grid, 14 cycles, 30 qubits, 2^10 slices, headline scheme as two "
                       "stems joined at the root, FP32", "n_tensors": len(order)}
    for name, (_, h, flops) in (("best_cut", best), ("early_cut", deep)):
        left, right, op = planner.two_sided_networks(pb, order, sliced, h, max_branch_rank=mbr)
        pl, pr = Plan(left), Plan(right)
        g = min(pl.default_slices_in_flight(n), pr.default_slices_in_flight(n))
        pl.tune(slices_in_flight=g, reps=2, cache_path=tune_cache)
        pr.tune(slices_in_flight=g, reps=2, cache_path=tune_cache)
        j = Join(pl, pr, op)
        res = j.contract(0, n, slices_in_flight=g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            j.contract(0, n, out=res, slices_in_flight=g)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        k = len(set(left["open_labels"]) & set(right["open_labels"]))
        err = float(np.linalg.norm(res.cpu().numpy()[0] - ref) / np.linalg.norm(ref))
        out[name] = {"cut": h, "shared_labels": k,
                     "left_peak_rank": pl.summary()["peak_rank"],
                     "right_peak_rank": pr.summary()["peak_rank"],
                     "ms_per_step": round(dt * 1e3, 3), "slices_per_s": round(n / dt, 1),
                     "tflops": round(flops * n / dt / 1e12, 2), "rel_l2_vs_one_sided": err}
        log(f"two-sided 30-qubit plan, cut {h} of {len(order)} ({k} shared labels): "
            f"{n / dt:.0f} slices/s, rel L2 vs one-sided {err:.2e}")
        j.close()
        pl.close()
        pr.close()
    return out


def merged14_30q(steps: int, tune_cache=None):
    """The headline circuit, order and sliced labels with branches merged up
    to 14 labels (the planner's default) instead of the 12 that keep every
    branch within 2^12 entries: fewer, larger products that move fewer
    bytes per slice."""
    import torch

    from paper_2005_06787_amd import Plan, planner
    from workloads import configs

    cfg = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]
    circ, oq, closed = configs.circuit_case(cfg)
    net = planner.plan_circuit(circ, oq, closed, n_sliced=cfg["n_sliced"], trials=64, seed=0,
                               max_branch_rank=14)
    out = {"workload": "5x6 grid, 14 cycles, 30 qubits, 2^10 slices, branches merged up to "
                       "2^14 entries"}
    for precision in ("fp32", "split_fp16"):
        plan = Plan(net, precision=precision)
        summ = plan.summary()
        n = int(summ["n_slices"])
        plan.tune(slices_in_flight=plan.default_slices_in_flight(n), reps=2, cache_path=tune_cache)
        res = plan.contract(0, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.contract(0, n, out=res)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[precision] = {"ms_per_step": round(dt * 1e3, 3), "slices_per_s": round(n / dt, 1),
                          "tflops": round(summ["flops_per_slice"] * n / dt / 1e12, 2)}
        log(f"30-qubit plan merged to 2^14 {precision}: {n / dt:.0f} slices/s")
        plan.close()
    out.update({"peak_rank": summ["peak_rank"], "n_steps": summ["n_steps"],
                "flops_per_slice": summ["flops_per_slice"],
                "bytes_per_slice": summ["bytes_per_slice"]})
    return out


def sampling_30q(n_prefixes: int, tune_cache=None):
    """Frugal rejection sampling on the 30-qubit, 14-cycle circuit: random
    prefixes of the 24 closed qubits as projected batch entries (64
    amplitudes each, all 2^10 slices), acceptance min(1, 2^n p / 10)."""
    import torch

    from paper_2005_06787_amd import Plan, planner, sampling
    from workloads import configs

    cfg = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]
    circ, oq, _ = configs.circuit_case(cfg)
    n = circ["n_qubits"]
    closed_q = [q for q in range(n) if q not in oq]
    net = planner.plan_circuit(circ, oq, None, closed_q, n_sliced=cfg["n_sliced"], trials=64,
                               seed=0, max_branch_rank=cfg["max_branch_rank"])
    plan = Plan(net)
    plan.tune(slices_in_flight=plan.default_slices_in_flight(1 << plan.n_sliced), reps=2,
              cache_path=tune_cache)
    prefixes = np.random.Generator(np.random.PCG64(4001)).integers(0, 1 << len(closed_q),
                                                                    n_prefixes)
    plan.contract(proj=prefixes[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sampling.sample(plan, n, oq, closed_q, prefixes, 10.0,
                          np.random.Generator(np.random.PCG64(4002)))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.close()
    log(f"sampling: {n_prefixes} batches in {dt:.2f} s, {res['n_samples']} samples, "
        f"XEB {res['xeb']:.3f}")
    return {"workload": f"30 qubits, 14 cycles, {n_prefixes} random prefixes of the 24 closed "
                        f"qubits x 64 open amplitudes, 2^10 slices each, M = 10, FP32",
            "batches_per_s": round(n_prefixes / dt, 3),
            "samples_per_s": round(res["n_samples"] / dt, 2),
            "acceptance": round(res["acceptance"], 4), "samples": res["n_samples"],
            "xeb_of_samples": round(res["xeb"], 4)}


def real_embedding_rate(plan, tune_log, steps, warmup, n_slices, stream):
    """The FP32 headline with every product computed as the real embedding
    (four real products per complex one) instead of the tuner's 3M choices:
    each such step takes its fastest real-embedding schedule from the
    tuning log.  Run after the headline numbers; the plan keeps these
    schedules."""
    best = {}
    with open(tune_log) as f:
        for ln in f:
            p = ln.split()
            if len(p) != 14 or p[0] != "stem-tune-v2" or p[12] != "0":
                continue
            key = tuple(int(x) for x in p[1:8])
            us = float(p[13])
            if key not in best or us < best[key][0]:
                best[key] = (us, [int(x) for x in p[8:12]])
    g = plan.default_slices_in_flight(n_slices)
    changed = 0
    for i, st in enumerate(plan.steps()):
        if st["sched_algo"] != 1:
            continue
        key = (0, st["amode"], st["cmode"], int(st["M"]).bit_length() - 1,
               int(st["K"]).bit_length() - 1, int(st["N"]).bit_length() - 1, g << st["n_batch"])
        if key not in best:
            return None
        tm, ntw, blocks, lds = best[key][1]
        plan.set_schedule(i, tm, ntw, blocks, lds, 0)
        changed += 1
    dt, _ = timed_run(plan, steps, warmup, n_slices, stream)
    ms = dt / steps * 1e3
    flops = plan.summary()["flops_per_slice"] * n_slices
    return {"ms_per_step": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 4),
            "slices_per_s": round(n_slices / (ms * 1e-3), 2), "steps_changed": changed}


def timed_run(plan, steps, warmup, n_slices, stream):
    import torch

    out = torch.empty((1, 1 << plan.n_open), dtype=torch.complex128, device="cuda")
    for _ in range(warmup):
        plan.contract(0, n_slices, out=out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        # per-kernel hipEvents on the last slice of the last step only
        plan.contract(0, n_slices, out=out, stream=stream, time_steps=(k == steps - 1))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, out


def roofline(plan):
    """Dominant kernel (the product) from the hipEvents of the last timed call.

    One product launch covers ``last_slices`` slices of one step; its
    algorithmic bytes are that many times the step's 8 (MK + MN + KN).
    """
    steps = plan.steps()
    nz = steps[0]["last_slices"]
    g_bytes = nz * sum(s["bytes"] for s in steps)
    g_flops = nz * sum(s["flops"] for s in steps)
    g_us = sum(s["last_gemm_us"] for s in steps)
    p_bytes = nz * sum(s["perm_bytes"] for s in steps)
    p_us = sum(s["last_perm_us"] for s in steps if s["permuted"])
    launches = len(steps)
    achieved = g_bytes / (g_us * 1e-6) / 1e9
    # every launch on its own roofline: max(bytes / 8 TB/s, flops / 157.3 TFLOP/s)
    roof_us = sum(max(nz * s["bytes"] / (HBM_PEAK_GBS * 1e9), nz * s["flops"] / FP32_PEAK_FLOPS)
                  for s in steps) * 1e6
    return {
        "kernel": "FP32 product launches (stem_cgemm_f32_kernel, stem_cgemm_f32g_kernel)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": recorded_traffic(g_bytes / launches),
        "slices_per_launch": nz,
        "bytes_per_launch": g_bytes / launches,
        "avg_launch_us": g_us / launches,
        "product_tflops": round(g_flops / (g_us * 1e-6) / 1e12, 3),
        "stepwise": {"roofline_us": round(roof_us, 1), "measured_us": round(g_us, 1),
                     "frac": round(roof_us / g_us, 4),
                     "note": "sum over the launches of max(bytes / 8 TB/s, flops / 157.3 "
                             "TFLOP/s), datasheet peaks, over their measured sum"},
        "permute": {"achieved_gbs": round(p_bytes / (p_us * 1e-6) / 1e9, 1) if p_us > 0 else None,
                    "bytes_per_group": p_bytes, "us_per_group": p_us},
    }


def cross_slice_kappa(plan, n_slices):
    """How much the slices cancel: sum_s |T_s| / |sum_s T_s|, over the whole
    amplitude vector (L2 norms) and per amplitude (median, max), from the
    per-slice results.  The amplitude error scales with it."""
    import torch

    per = torch.stack([plan.contract(s, s + 1)[0] for s in range(n_slices)]).cpu().numpy()
    tot = per.sum(axis=0)
    vec = float(np.linalg.norm(per, axis=1).sum() / np.linalg.norm(tot))
    amp = np.abs(per).sum(axis=0) / np.maximum(np.abs(tot), 1e-300)
    return {"vector": round(vec, 3), "amplitude_median": round(float(np.median(amp)), 3),
            "amplitude_max": round(float(amp.max()), 3)}


def cpu_baseline(net, sample_slices, flops_per_slice):
    """The FP64 oracle, as it stands, on a few slices (host cores)."""
    from oracle import stemnet

    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    onet = dict(net)
    onet["stem"] = {"labels": net["stem"]["labels"],
                    "data": np.asarray(net["stem"]["data"], np.complex128)}
    onet["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                        for b in net["branches"]]
    refs = {}
    t0 = time.perf_counter()
    for s in sample_slices:
        v, _ = stemnet.run_slice(onet, int(s))
        refs[int(s)] = v.reshape(-1)
    dt = time.perf_counter() - t0
    rate = len(sample_slices) / dt
    return {"value": round(rate * flops_per_slice / 1e12, 6), "unit": "TFLOP/s",
            "slices_per_s": round(rate, 4), "cores": int(cores), "kind": "oracle",
            "sample": f"{len(sample_slices)} slices of the 2^10 (FP64 plan-following "
                      f"contraction, {dt:.1f} s)"}, refs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-split", action="store_true", help="skip the split-FP16 run")
    ap.add_argument("--no-tune", action="store_true", help="default launch schedules")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the comparison runs (FP32 real embedding) and the other workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy and exit (counter calibration)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache / measurement log")
    args = ap.parse_args()
    if args.copy_calibration:
        # one plain device-to-device copy of 1 GiB, to calibrate the HBM
        # traffic counters (FETCH_SIZE / WRITE_SIZE) against a known size
        import torch

        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30}))
        return
    if args.tune_cache is None:
        # the tuner's measurement log, also read back for the real-embedding rate
        import tempfile

        args.tune_cache = os.path.join(tempfile.mkdtemp(prefix="stem_tune_"), "tune.txt")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "layout is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch

    from oracle import stats
    from paper_2005_06787_amd import Plan

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    net, cfg = make_net()
    log(f"plan made in {time.perf_counter() - t0:.1f} s: "
        f"{ {k: v for k, v in net['stats'].items() if k != 'order'} }")
    stream = torch.cuda.current_stream()

    results = {}
    plans = {}
    for precision in (["fp32"] if args.no_split else ["fp32", "split_fp16"]):
        plan = Plan(net, precision=precision)
        summ = plan.summary()
        n_slices = summ["n_slices"]
        if not args.no_tune:
            t0 = time.perf_counter()
            plan.tune(slices_in_flight=plan.default_slices_in_flight(n_slices), reps=3,
                      cache_path=args.tune_cache)
            log(f"{precision}: schedules tuned in {time.perf_counter() - t0:.1f} s")
        dt, out = timed_run(plan, args.steps, args.warmup, n_slices, stream)
        ms = dt / args.steps * 1e3
        flops = summ["flops_per_slice"] * n_slices
        results[precision] = {
            "ms_per_step": ms,
            "tflops": flops / (ms * 1e-3) / 1e12,
            "slices_per_s": n_slices / (ms * 1e-3),
            "amps": out.cpu().numpy()[0],
            "summary": summ,
        }
        plans[precision] = plan
        log(f"{precision}: {ms:.2f} ms per step ({n_slices} slices), "
            f"{results[precision]['tflops']:.3f} TFLOP/s, "
            f"{results[precision]['slices_per_s']:.1f} slices/s")

    fp32 = results["fp32"]
    summ = fp32["summary"]
    line = {
        "metric": "stem contraction TFLOP/s & slices/s, split-FP16 vs FP32, at 1e-5 amp error",
        "value": round(fp32["tflops"], 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp32["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "5x6 grid, 14 cycles, 30 qubits, 6 open (64 amplitudes), "
                               "2^10 slices, branches of 2^4-2^12 entries, FP32 complex "
                               "products",
                   "n_slices": summ["n_slices"], "n_steps": summ["n_steps"],
                   "peak_rank": summ["peak_rank"], "n_permutes": summ["n_permutes"],
                   "parallelism": "1 GPU"},
        "slices_per_s": round(fp32["slices_per_s"], 2),
        "flops_per_slice": summ["flops_per_slice"],
        "bytes_per_slice": summ["bytes_per_slice"],
        "roofline": roofline(plans["fp32"]),
    }
    if "split_fp16" in results:
        sp = results["split_fp16"]
        line["split_fp16"] = {"value": round(sp["tflops"], 4), "unit": "TFLOP/s",
                              "slices_per_s": round(sp["slices_per_s"], 2),
                              "ms_per_step": round(sp["ms_per_step"], 3)}
    # amplitude error: sampled slices against the FP64 oracle (also the CPU baseline)
    if not args.no_cpu:
        rng = np.random.Generator(np.random.PCG64(cfg["slice_sample_seed"]))
        sample = [int(s) for s in rng.choice(summ["n_slices"], size=64, replace=False)]
        base, refs = cpu_baseline(net, sample, summ["flops_per_slice"])
        line["cpu_baseline"] = base
        errs = {}
        for precision, plan in plans.items():
            worst = 0.0
            for s in sample[:4]:
                got = plan.contract(s, s + 1).cpu().numpy()[0]
                worst = max(worst, stats.rel_l2(got, refs[s]))
            errs[precision] = worst
        line["amp_rel_l2_vs_oracle"] = errs
        line["cross_slice_kappa"] = cross_slice_kappa(plans["fp32"], summ["n_slices"])
    if not args.no_tune and not args.no_extra:
        re_ = real_embedding_rate(plans["fp32"], args.tune_cache, args.steps, args.warmup,
                                  summ["n_slices"], stream)
        if re_ is not None:
            line["fp32_real_embedding"] = re_
    for p in plans.values():
        p.close()
    torch.cuda.empty_cache()
    if not args.no_extra:
        line["isolated_stem_2e30"] = isolated_stem(3, args.tune_cache)
        line["batched_8_circuits"] = batched_workload(3, args.tune_cache)
        line["slice_53q_m20"] = slice_53q(3, args.tune_cache)
        line["sampling_30q"] = sampling_30q(8, args.tune_cache)
        line["locally_optimised_30q"] = locally_optimised_30q(3, args.tune_cache)
        line["merged14_30q"] = merged14_30q(3, args.tune_cache)
        line["two_sided_30q"] = two_sided_30q(3, args.tune_cache)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
