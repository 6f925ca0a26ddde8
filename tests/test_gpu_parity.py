"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Every network here is small enough for the oracle to finish in seconds,
yet spans several 64-row tiles of the product kernel, ragged K/N (K or N
below the 16-wide MFMA tile), steps with and without a stem permute,
sliced labels on the stem and on branches, and projected labels.

Tolerances: FP32 and split-FP16 products, relative L2 <= 1e-5 over every
result vector (the benchmark spec's bound).  Split-BF16 keeps 8 + 8 significant
bits per factor, so each product carries a relative error near 2^-16
(1.5e-5) of the *absolute* sum of its terms; over a dozen steps, and for a
scalar result where those terms cancel, the relative L2 error reaches a few
1e-4, so its bound is 5e-4 (it does not meet the 1e-5 target, by design).
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads import tensors as wt
from workloads.networks import random_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan, stem_fill_counter, stem_xeb_f64  # noqa: E402
from paper_2005_06787_amd import _capi as C  # noqa: E402

TOL = {"fp32": 1e-5, "split_fp16": 1e-5, "split_bf16": 5e-4}

NETS = [
    # (seed, stem_rank, n_steps, s_range, f_range, n_sliced, n_proj, n_open_final)
    (1, 8, 6, (1, 3), (0, 3), 2, 1, 5),
    (2, 12, 8, (1, 4), (1, 4), 3, 2, 6),
    (3, 14, 10, (2, 6), (2, 6), 2, 1, 8),
    (4, 10, 6, (0, 2), (0, 2), 1, 1, 4),     # outer products (s = 0) and f = 0
    (5, 16, 6, (4, 7), (4, 7), 2, 0, 10),    # K, N up to 128
    (6, 13, 12, (1, 3), (1, 3), 4, 1, 0),    # scalar result (n_open = 0)
    (7, 9, 5, (3, 5), (0, 1), 0, 3, 3),
    (8, 15, 8, (5, 8), (5, 8), 1, 1, 9),     # K, N up to 256: split over blockIdx.y
]


def _net(cfg):
    seed, r, n, sr, fr, nsl, npr, nof = cfg
    return random_stem_network(seed, stem_rank=r, n_steps=n, s_range=sr, f_range=fr,
                               n_sliced=nsl, n_proj=npr, n_open_final=nof,
                               rank_bounds=(1, r + 3))


def _oracle_net(net):
    """Oracle input: the same tensors, widened to complex128."""
    out = dict(net)
    out["stem"] = {"labels": net["stem"]["labels"],
                   "data": np.asarray(net["stem"]["data"], dtype=np.complex128)}
    out["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                       for b in net["branches"]]
    return out


@pytest.mark.parametrize("cfg", NETS, ids=lambda c: f"seed{c[0]}")
@pytest.mark.parametrize("precision", ["fp32", "split_fp16", "split_bf16"])
def test_per_slice_matches_oracle(cfg, precision):
    net = _net(cfg)
    onet = _oracle_net(net)
    print(f"network seed {cfg[0]} precision {precision}", flush=True)
    plan = Plan(net, precision=precision)
    n_sl, n_pr = len(net["sliced_labels"]), len(net["proj_labels"])
    projs = list(range(1 << n_pr))
    for s in range(1 << n_sl):
        got = plan.contract(s, s + 1, proj=projs).cpu().numpy()
        for p in projs:
            ref, _ = stemnet.run_slice(onet, s, p)
            err = stats.rel_l2(got[p], ref.reshape(-1))
            assert err <= TOL[precision], (s, p, err)
    plan.close()


@pytest.mark.parametrize("cfg", NETS[:4], ids=lambda c: f"seed{c[0]}")
def test_sliced_sum_and_accumulate(cfg):
    net = _net(cfg)
    onet = _oracle_net(net)
    plan = Plan(net)
    n_sl, n_pr = len(net["sliced_labels"]), len(net["proj_labels"])
    projs = list(range(1 << n_pr))
    full = plan.contract(0, 1 << n_sl, proj=projs)
    for p in projs:
        ref = stemnet.sliced_sum(onet, proj=p).reshape(-1)
        assert stats.rel_l2(full[p].cpu().numpy(), ref) <= 1e-5
    # two halves with STEM_ACCUMULATE give the same sum
    half = (1 << n_sl) // 2
    part = plan.contract(0, half, proj=projs)
    plan.contract(half, 1 << n_sl, proj=projs, out=part, accumulate=True)
    assert torch.allclose(part, full, rtol=1e-12, atol=1e-12)
    # deterministic: the same call twice gives identical bits
    again = plan.contract(0, 1 << n_sl, proj=projs)
    assert torch.equal(again, full)
    # empty range writes zeros
    z = plan.contract(1, 1, proj=projs)
    assert torch.count_nonzero(z).item() == 0
    # any number of slices per launch gives the same bits: every slice is
    # computed the same way and added in slice order
    for group in (1, 3, 1 << n_sl):
        g = plan.contract(0, 1 << n_sl, proj=projs, slices_in_flight=group)
        assert torch.equal(g, full), group
    plan.close()


def test_range_and_workspace_errors():
    net = _net(NETS[1])
    plan = Plan(net)
    n_sl = len(net["sliced_labels"])
    with pytest.raises(C.StemError) as e:
        plan.contract(0, (1 << n_sl) + 1)
    assert e.value.status == C.STEM_ERANGE
    with pytest.raises(C.StemError) as e:
        plan.contract(0, 1, proj=[1 << len(net["proj_labels"])])
    assert e.value.status == C.STEM_ERANGE
    out = torch.empty((1, 1 << plan.n_open), dtype=torch.complex128, device="cuda")
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    import ctypes
    st = C.lib().stem_contract(plan._h, 0, 1, None, 1, ctypes.c_void_p(small.data_ptr()), 256,
                               ctypes.c_void_p(out.data_ptr()), 0,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == C.STEM_ENOMEM
    with pytest.raises(C.StemError) as e:
        plan.workspace_bytes(0)
    assert e.value.status == C.STEM_ERANGE
    assert plan.workspace_bytes(8) == 8 * plan.workspace_bytes(1)
    plan.close()


def test_no_branch_plan_is_reorder_of_stem():
    rng = np.random.Generator(np.random.PCG64(11))
    data = (rng.standard_normal((2,) * 5) + 1j * rng.standard_normal((2,) * 5)).astype(np.complex64)
    net = {"open_labels": [4, 0, 2], "sliced_labels": [1], "proj_labels": [3],
           "stem": {"labels": [0, 1, 2, 3, 4], "data": data}, "branches": []}
    plan = Plan(net)
    got = plan.contract(0, 2, proj=[0, 1]).cpu().numpy()
    for p in range(2):
        ref = stemnet.sliced_sum(_oracle_net(net), proj=p).reshape(-1)
        assert stats.rel_l2(got[p], ref) <= 1e-6
    plan.close()


def test_fill_counter_bit_exact():
    n = 1 << 16
    t = torch.empty(n, dtype=torch.complex64, device="cuda")
    stem_fill_counter(t, seed=1234, scale_log2=30)
    ref = wt.counter_stem_entries(1234, np.arange(n), 30).astype(np.complex64)
    assert np.array_equal(t.cpu().numpy(), ref)


def test_isolated_stem_device_input():
    iso = wt.random_isolated_stem(18, 6, seed=3, s_range=(2, 5), r_range=(4, 9))
    r0 = len(iso["stem_labels"])
    stem = torch.empty(1 << r0, dtype=torch.complex64, device="cuda")
    stem_fill_counter(stem, iso["stem_seed"], iso["stem_scale_log2"])
    net = {"open_labels": iso["final_labels"], "sliced_labels": [], "proj_labels": [],
           "stem": {"labels": iso["stem_labels"]}, "branches": iso["branches"]}
    for precision in ("fp32", "split_fp16"):
        plan = Plan(net, precision=precision, stem_device=stem)
        got = plan.contract().cpu().numpy()[0]
        plan.close()
        ref_stem = wt.counter_stem_entries(iso["stem_seed"], np.arange(1 << r0),
                                           iso["stem_scale_log2"]).reshape((2,) * r0)
        onet = _oracle_net(dict(net, stem={"labels": iso["stem_labels"], "data": ref_stem}))
        ref, _ = stemnet.run_slice(onet, 0, 0)
        assert stats.rel_l2(got, ref.reshape(-1)) <= TOL[precision], precision


def test_xeb_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(5))
    n_q = 12
    a = (rng.standard_normal(3000) + 1j * rng.standard_normal(3000)) / np.sqrt(2 * 2 ** n_q)
    t = torch.from_numpy(a).cuda()
    out = stem_xeb_f64(t, n_q).cpu().numpy()
    assert abs(out[0] - stats.xeb(a, n_q)) <= 1e-12 * max(1.0, abs(stats.xeb(a, n_q)))
    assert abs(out[1] - np.sum(np.abs(a) ** 2)) <= 1e-12
