"""Two stems joined at the root (paper §A.2) through the C-ABI join.

Random stem networks are cut into a left stem (the stem and the first
branches) and a right stem (the other branches, the first of them as its
initial stem); both halves run as plans and the join contracts their final
tensors over the shared labels.  Compared with the FP64 oracle's
``join_slice`` per slice and projected assignment (FP32 and split FP16 at
relative L2 <= 1e-5), with the network's one-sided value, across cuts
with and without steps on either side, a scalar result, shared index
lengths from 1 to several k chunks, hyperedges, groups of slices per
launch (bit-identical) and the label errors of the join.
"""
import ctypes

import numpy as np
import pytest

from oracle import stats, stemnet
from workloads.networks import random_stem_network, split_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Join, Plan  # noqa: E402
from paper_2005_06787_amd import _capi as C  # noqa: E402

NETS = [
    # (seed, stem_rank, n_steps, s_range, f_range, n_sliced, n_proj, n_open_final, batch_prob)
    (31, 12, 8, (1, 4), (0, 4), 2, 1, 6, 0.0),
    (32, 16, 10, (1, 5), (0, 5), 2, 1, 8, 0.0),    # shared index up to 2^16: several k chunks
    (33, 10, 8, (1, 3), (0, 3), 3, 2, 4, 0.4),     # hyperedges
    (34, 14, 8, (2, 5), (1, 5), 1, 0, 0, 0.0),     # scalar result
    (35, 20, 6, (2, 6), (2, 6), 1, 1, 6, 0.0),     # shared index near 2^20
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


def _cuts(net):
    n = len(net["branches"])
    out = []
    for h in sorted({1, n // 2, n - 1}):
        try:
            out.append((h,) + split_stem_network(net, h))
        except ValueError:
            pass
    return out


@pytest.mark.parametrize("cfg", NETS, ids=lambda c: f"seed{c[0]}")
@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_join_matches_oracle(cfg, precision):
    net = _net(cfg)
    cuts = _cuts(net)
    assert cuts, "no valid cut"
    n_sl, n_pr = len(net["sliced_labels"]), len(net["proj_labels"])
    projs = list(range(1 << n_pr))
    whole = _c128(net)
    for h, left, right in cuts:
        print(f"network seed {cfg[0]} cut {h} precision {precision}", flush=True)
        pl, pr = Plan(left, precision=precision), Plan(right, precision=precision)
        j = Join(pl, pr, net["open_labels"])
        ol, orr = _c128(left), _c128(right)
        for s in range(1 << n_sl):
            got = j.contract(s, s + 1, proj=projs).cpu().numpy()
            for p in projs:
                ref = stemnet.join_slice(ol, orr, net["open_labels"], s, p).reshape(-1)
                err = stats.rel_l2(got[p], ref)
                assert err <= 1e-5, (h, s, p, err)
        tot = j.contract(proj=projs).cpu().numpy()
        for p in projs:
            ref = stemnet.sliced_sum(whole, proj=p).reshape(-1)
            assert stats.rel_l2(tot[p], ref) <= 1e-5, (h, p)
        j.close()
        pl.close()
        pr.close()


@pytest.mark.parametrize("cfg", NETS[:2], ids=lambda c: f"seed{c[0]}")
def test_join_groups_bit_identical(cfg):
    net = _net(cfg)
    h, left, right = _cuts(net)[-1]
    pl, pr = Plan(left), Plan(right)
    j = Join(pl, pr, net["open_labels"])
    n = 1 << pl.n_sliced
    one = j.contract(0, n, slices_in_flight=1)
    many = j.contract(0, n, slices_in_flight=n).clone()
    acc = j.contract(0, 1)
    j.contract(1, n, out=acc, accumulate=True)
    assert torch.equal(one, many)
    assert stats.rel_l2(acc.cpu().numpy(), many.cpu().numpy()) <= 1e-14
    j.close()


def test_join_without_steps_and_same_plan():
    """Stems with no branches (the final tensors are the stems' slices) and
    one plan used as both halves (every label shared: a scalar)."""
    rng = np.random.Generator(np.random.PCG64(9))

    def rnd(rank):
        return (rng.standard_normal((2,) * rank) + 1j * rng.standard_normal((2,) * rank)
                ).astype(np.complex64)

    left = {"open_labels": [0, 1, 2, 3, 4, 5, 6, 7, 8, 9], "sliced_labels": [20, 21],
            "proj_labels": [30], "stem": {"labels": [0, 20, 1, 2, 3, 4, 30, 5, 6, 7, 8, 9],
                                          "data": rnd(12)}, "branches": []}
    right = {"open_labels": [9, 8, 7, 6, 5, 4, 3, 2, 1, 40, 41], "sliced_labels": [20, 21],
             "proj_labels": [30], "stem": {"labels": [9, 8, 21, 7, 6, 5, 4, 3, 2, 1, 40, 41],
                                           "data": rnd(12)}, "branches": []}
    pl, pr = Plan(left), Plan(right)
    j = Join(pl, pr, [41, 0, 40])
    got = j.contract(proj=[0, 1]).cpu().numpy()
    for p in (0, 1):
        ref = stemnet.join_sliced_sum(_c128(left), _c128(right), [41, 0, 40], proj=p)
        assert stats.rel_l2(got[p], ref.reshape(-1)) <= 1e-6
    j.close()
    jj = Join(pl, pl, [])
    got = jj.contract(proj=[1]).cpu().numpy()
    ref = stemnet.join_sliced_sum(_c128(left), _c128(left), [], proj=1)
    assert stats.rel_l2(got[0], ref.reshape(-1)) <= 1e-6
    jj.close()


def test_join_label_errors():
    net = _net(NETS[0])
    h, left, right = _cuts(net)[0]
    pl, pr = Plan(left), Plan(right)
    with pytest.raises(C.StemError) as e:
        Join(pl, pr, net["open_labels"][1:])
    assert e.value.status == C.STEM_ELABEL
    other = dict(right, sliced_labels=list(reversed(right["sliced_labels"])))
    po = Plan(other)
    with pytest.raises(C.StemError) as e:
        Join(pl, po, net["open_labels"])
    assert e.value.status == C.STEM_ELABEL
    j = Join(pl, pr, net["open_labels"])
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = torch.empty(1 << len(net["open_labels"]), dtype=torch.complex128, device="cuda")
    st = C.lib().stem_join_contract(j._h, 0, 1, None, 1, ctypes.c_void_p(ws.data_ptr()), 16,
                                    ctypes.c_void_p(out.data_ptr()), 0, None)
    assert st == C.STEM_ENOMEM
    st = C.lib().stem_join_contract(j._h, 0, 1, None, 1, ctypes.c_void_p(ws.data_ptr()), 16,
                                    ctypes.c_void_p(out.data_ptr()), C.STEM_TIME_STEPS, None)
    assert st == C.STEM_EINVAL
    j.close()


def test_two_sided_circuit_plan_matches_oracle():
    """A circuit's scheme cut into two stems meeting at the root (4x5 grid,
    8 cycles, 6 open qubits, 2^4 slices): the GPU join equals the oracle's
    join of the same two networks, and the one-sided plan's amplitudes."""
    from paper_2005_06787_amd import planner
    from workloads import circuits as wc
    from workloads import tensors as wt

    c = wc.make_circuit(4, 5, 8, seed=1)
    open_q = wc.block_qubits(4, 5, range(0, 2), range(2, 5))
    pre = wt.split_open_prefix(20, open_q, 1001)
    closed = dict(zip(pre["closed"], pre["closed_bits"]))
    pb = planner.CircuitProblem(c, open_q, closed)
    order, sliced, _, _ = planner.find_scheme(pb.tlabels, 8, 0, n_sliced=4, forbid=pb.forbid)
    one = planner.scheme_network(pb, order, sliced)
    p1 = Plan(one)
    ref_one = p1.contract().cpu().numpy()[0]
    p1.close()
    m = len(order)
    for h in (m // 3, m // 2, m - 3):
        left, right, op = planner.two_sided_networks(pb, order, sliced, h)
        print(f"circuit cut {h} of {m}", flush=True)
        pl, pr = Plan(left), Plan(right)
        j = Join(pl, pr, op)
        got = j.contract().cpu().numpy()[0]
        ref = stemnet.join_sliced_sum(_c128(left), _c128(right), op).reshape(-1)
        assert stats.rel_l2(got, ref) <= 1e-5, h
        assert stats.rel_l2(got, ref_one) <= 1e-5, h
        j.close()
        pl.close()
        pr.close()
