"""Slice ranges of several circuits as one HIP graph (C-ABI stem_batch_*).

Three seeded 4x5-grid circuits with different depths and sliced-label
counts run as one graph with one chain per circuit.  Every replay must give
the same bits as stem_contract on each plan alone (slices are added in
slice order either way), also with other GPU work between replays, and one
circuit's amplitudes must match the FP64 state vector (relative L2 <= 1e-5).
"""
import numpy as np
import pytest

from oracle import stats, statevector
from paper_2005_06787_amd import Batch, Plan, planner
from paper_2005_06787_amd import _capi as C
from workloads import configs, tensors
from workloads.circuits import make_circuit

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CIRCUITS = [(6, 10, 3), (8, 11, 5), (10, 12, 6)]  # (cycles, seed, sliced labels)


@pytest.fixture(scope="module")
def nets():
    cfg = configs.CIRCUIT_CONFIGS["c1_4x5_m8"]
    oq = configs.open_qubits(cfg)
    out = []
    for cycles, seed, nsl in CIRCUITS:
        circ = make_circuit(4, 5, cycles, seed)
        pre = tensors.split_open_prefix(20, oq, seed + 1000)
        closed = dict(zip(pre["closed"], pre["closed_bits"]))
        net = planner.plan_circuit(circ, oq, closed, n_sliced=nsl, trials=8, seed=0)
        out.append((circ, pre, net))
    return out


def test_batch_graph_matches_contract_and_oracle(nets):
    plans = [Plan(net) for _, _, net in nets]
    ranges = [(0, 1 << p.n_sliced) for p in plans]
    eager = [p.contract(a, b)[0].clone() for p, (a, b) in zip(plans, ranges)]
    batch = Batch(plans, ranges)
    for rep in range(3):
        outs = batch.launch()
        torch.cuda.synchronize()
        for j, o in enumerate(outs):
            assert torch.equal(o, eager[j]), (rep, j)
        # other GPU work between replays
        plans[0].contract(0, 1)
        x = torch.randn(1 << 16, device="cuda")
        (x * 2).sum().item()
    # the first circuit against the state vector
    circ, pre, _ = nets[0]
    psi = statevector.run(circ)
    ref = statevector.batch_amplitudes(psi, 20, pre["open"], pre["closed"], pre["closed_bits"])
    assert stats.rel_l2(batch.outs[0].cpu().numpy(), ref) <= 1e-5
    batch.close()
    for p in plans:
        p.close()


def test_batch_accumulate_and_sub_ranges(nets):
    plans = [Plan(net) for _, _, net in nets[:2]]
    ranges = [(1, 5), (2, 2)]   # a partial range and an empty one
    eager = [p.contract(a, b)[0].clone() for p, (a, b) in zip(plans, ranges)]
    outs = [torch.zeros(1 << p.n_open, dtype=torch.complex128, device="cuda") for p in plans]
    batch = Batch(plans, ranges, outs=outs, accumulate=True)
    batch.launch()
    batch.launch()
    torch.cuda.synchronize()
    for o, e in zip(outs, eager):
        assert torch.allclose(o, 2 * e, rtol=1e-14, atol=0)
    batch.close()
    for p in plans:
        p.close()


def test_batch_errors(nets):
    plan = Plan(nets[2][2])
    assert plan.summary()["n_steps"] > 0   # so a workspace is needed
    with pytest.raises(C.StemError) as e:
        Batch([plan], [(0, (1 << plan.n_sliced) + 1)])
    assert e.value.status == C.STEM_ERANGE
    with pytest.raises(C.StemError) as e:
        Batch([plan], [(0, 1)], ws_bytes=256)
    assert e.value.status == C.STEM_ENOMEM
    plan.close()
