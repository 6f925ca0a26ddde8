"""Circuit workloads end to end on the GPU against the FP64 oracle.

4x5 grid, 8 cycles (20 qubits): amplitudes from the stem contraction equal
the state-vector amplitudes (relative L2 <= 1e-5), for 64 uniform
bitstrings (every qubit projected, scalar results), for the 6-open-qubit
batch with a seeded prefix, and for all 2^20 amplitudes as 2^14 projected
prefixes; their total probability is 1 and the XEB of bitstrings sampled
from the ideal distribution matches the oracle's.  The sliced-sum identity
is checked at this size against the state vector.  The 5x6 grid, 14
cycles (30 qubits, 2^10 slices) is checked slice by slice on sampled slices
against the FP64 plan-following oracle.
"""
import numpy as np
import pytest

from oracle import stats, statevector, stemnet
from paper_2005_06787_amd import Plan, planner, stem_xeb_f64
from workloads import configs, tensors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C1 = configs.CIRCUIT_CONFIGS["c1_4x5_m8"]
C2 = configs.CIRCUIT_CONFIGS["c2_5x6_m14"]


def _c128(net):
    out = dict(net)
    out["stem"] = {"labels": net["stem"]["labels"],
                   "data": np.asarray(net["stem"]["data"], np.complex128)}
    out["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                       for b in net["branches"]]
    return out


@pytest.fixture(scope="module")
def c1():
    from workloads.circuits import make_circuit

    circ = make_circuit(C1["rows"], C1["cols"], C1["cycles"], C1["seed"])
    psi = statevector.run(circ)
    return circ, psi


def test_c1_uniform_bitstrings(c1):
    circ, psi = c1
    n = circ["n_qubits"]
    bits = tensors.random_bitstrings(n, 64, C1["bitstring_seed"])
    net = planner.plan_circuit(circ, [], None, list(range(n)), n_sliced=0, trials=8, seed=0)
    plan = Plan(net)
    got = plan.contract(proj=bits).cpu().numpy()[:, 0]
    plan.close()
    ref = statevector.amplitudes(psi, bits)
    print("c1 uniform bitstrings rel L2", stats.rel_l2(got, ref))
    assert stats.rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("precision,n_sliced", [("fp32", 0), ("fp32", 6), ("split_fp16", 3)])
def test_c1_open_batch_and_sliced_sum(c1, precision, n_sliced):
    circ, psi = c1
    oq = configs.open_qubits(C1)
    pre = tensors.split_open_prefix(circ["n_qubits"], oq, C1["prefix_seed"])
    closed = dict(zip(pre["closed"], pre["closed_bits"]))
    net = planner.plan_circuit(circ, oq, closed, n_sliced=n_sliced, trials=8, seed=0)
    plan = Plan(net, precision=precision)
    got = plan.contract().cpu().numpy()[0]
    plan.close()
    ref = statevector.batch_amplitudes(psi, circ["n_qubits"], oq, pre["closed"],
                                       pre["closed_bits"])
    print(precision, n_sliced, "rel L2", stats.rel_l2(got, ref))
    assert stats.rel_l2(got, ref) <= 1e-5


def test_c1_all_amplitudes_norm_and_xeb(c1):
    circ, psi = c1
    n = circ["n_qubits"]
    oq = configs.open_qubits(C1)
    closed_q = [q for q in range(n) if q not in oq]
    net = planner.plan_circuit(circ, oq, None, closed_q, n_sliced=0, trials=8, seed=0)
    plan = Plan(net)
    prefixes = list(range(1 << len(closed_q)))
    amps = plan.contract(proj=prefixes)          # [2^14, 2^6], open qubits inner
    plan.close()
    got = amps.cpu().numpy()
    # reorder the oracle's vector to (closed bits, open bits)
    t = psi.reshape((2,) * n)
    ref = np.transpose(t, closed_q + oq).reshape(len(prefixes), -1)
    assert stats.rel_l2(got, ref) <= 1e-5
    xs = stem_xeb_f64(amps.reshape(-1), n).cpu().numpy()
    assert abs(xs[1] - 1.0) <= 1e-5                       # total probability
    # XEB over bitstrings sampled from the ideal distribution (paper §2)
    p = np.abs(psi) ** 2
    rng = np.random.Generator(np.random.PCG64(C1["sample_seed"]))
    sample = rng.choice(p.size, size=4096, p=p / p.sum())
    flat = amps.reshape(-1)
    # index of bitstring x in the (closed, open) order of the GPU result
    bits = ((sample[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1)
    order = closed_q + oq
    idx = np.zeros(len(sample), dtype=np.int64)
    for q in order:
        idx = (idx << 1) | bits[:, q]
    sel = flat[torch.from_numpy(idx).cuda()].contiguous()
    xeb_gpu = stem_xeb_f64(sel, n).cpu().numpy()[0]
    xeb_ref = stats.xeb(psi[sample], n)
    print("XEB gpu", xeb_gpu, "oracle", xeb_ref)
    assert abs(xeb_gpu - xeb_ref) <= 1e-5 * abs(xeb_ref)
    assert 0.75 < xeb_ref < 1.25


@pytest.fixture(scope="module")
def c2_plan():
    from workloads.circuits import make_circuit

    circ = make_circuit(C2["rows"], C2["cols"], C2["cycles"], C2["seed"])
    oq = configs.open_qubits(C2)
    pre = tensors.split_open_prefix(circ["n_qubits"], oq, C2["prefix_seed"])
    closed = dict(zip(pre["closed"], pre["closed_bits"]))
    return planner.plan_circuit(circ, oq, closed, n_sliced=C2["n_sliced"], trials=64, seed=0,
                                max_branch_rank=C2["max_branch_rank"])


@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_c2_sampled_slices(c2_plan, precision):
    net = c2_plan
    plan = Plan(net, precision=precision)
    summ = plan.summary()
    print("c2 plan", summ, flush=True)
    assert summ["n_slices"] == 1 << C2["n_sliced"]
    rng = np.random.Generator(np.random.PCG64(C2["slice_sample_seed"]))
    onet = _c128(net)
    for s in rng.choice(summ["n_slices"], size=2, replace=False):
        got = plan.contract(int(s), int(s) + 1).cpu().numpy()[0]
        ref, _ = stemnet.run_slice(onet, int(s))
        err = stats.rel_l2(got, ref.reshape(-1))
        print("slice", s, precision, "rel L2", err, flush=True)
        assert err <= 1e-5
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "split_fp16"])
def test_c2_full_size_in_the_bench_launch_configuration(c2_plan, precision, tmp_path):
    """All 2^10 slices in the launch configuration bench.py times (its
    slices per launch, tuned schedules) equal, bit for bit, the same slices
    contracted one per launch and added in slice order; sampled single
    slices match the oracle (test_c2_sampled_slices), so the full-size sum
    does too."""
    plan = Plan(c2_plan, precision=precision)
    n = int(plan.summary()["n_slices"])
    group = plan.default_slices_in_flight(n)
    plan.tune(slices_in_flight=group, reps=1, cache_path=str(tmp_path / "tune.txt"))
    full = plan.contract(0, n, slices_in_flight=group)
    one = torch.zeros_like(full)
    for s in range(n):
        plan.contract(s, s + 1, out=one, accumulate=True, slices_in_flight=1)
    torch.cuda.synchronize()
    print(precision, "slices per launch", group, flush=True)
    assert torch.equal(full, one)
    plan.close()
