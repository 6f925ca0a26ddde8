"""Frugal rejection sampling end to end on the 20-qubit, 8-cycle circuit
(paper §3): 256 random prefixes of the 14 closed qubits go through one
contraction as projected batch entries (64 amplitudes each), candidates
are accepted with probability min(1, 2^n p / M), M = 10.

Checked against the FP64 state vector: the produced bitstrings' GPU
amplitudes equal the oracle's; the acceptance rate and the XEB of the
produced samples equal the oracle's expectations for this M
(stats.frugal_acceptance, stats.frugal_xeb) within 5 standard errors;
one sample per batch in the 'first' mode, for at least 95 % of batches.
"""
import numpy as np
import pytest

from oracle import stats, statevector
from workloads import circuits as wc
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan, planner, sampling  # noqa: E402

C1 = configs.CIRCUIT_CONFIGS["c1_4x5_m8"]
M = 10.0


@pytest.fixture(scope="module")
def setup():
    circ = wc.make_circuit(C1["rows"], C1["cols"], C1["cycles"], C1["seed"])
    n = circ["n_qubits"]
    psi = statevector.run(circ)
    oq = configs.open_qubits(C1)
    closed_q = [q for q in range(n) if q not in oq]
    plan = Plan(planner.plan_circuit(circ, oq, None, closed_q, n_sliced=0, trials=8, seed=0))
    prefixes = np.random.Generator(np.random.PCG64(3001)).integers(0, 1 << len(closed_q), 256)
    yield n, psi, oq, closed_q, plan, prefixes
    plan.close()


def test_samples_match_the_state_vector(setup):
    n, psi, oq, closed_q, plan, prefixes = setup
    res = sampling.sample(plan, n, oq, closed_q, prefixes, M, np.random.Generator(np.random.PCG64(3002)))
    x = res["bitstrings"]
    got = res["amplitudes"].cpu().numpy()
    assert stats.rel_l2(got, psi[x]) <= 1e-5
    assert res["xeb"] == pytest.approx(stats.xeb(got, n), abs=1e-12)
    p_all = np.abs(psi) ** 2
    # acceptance: per-batch fractions give the standard error
    probs = np.abs(plan.contract(proj=prefixes).cpu().numpy()) ** 2
    frac = np.minimum(1.0, (2.0 ** n) * probs / M).mean(axis=1)
    want_acc = stats.frugal_acceptance(p_all, M)
    se_acc = frac.std(ddof=1) / np.sqrt(len(frac)) + 1.0 / np.sqrt(res["candidates"])
    want_xeb = stats.frugal_xeb(p_all, M)
    npx = (2.0 ** n) * np.abs(got) ** 2
    se_xeb = npx.std(ddof=1) / np.sqrt(len(npx))
    print(f"{res['candidates']} candidates, {res['n_samples']} samples: acceptance "
          f"{res['acceptance']:.4f} (expected {want_acc:.4f}), XEB {res['xeb']:.3f} "
          f"(expected {want_xeb:.3f} +- {se_xeb:.3f})")
    assert abs(res["acceptance"] - want_acc) <= 5 * se_acc
    assert abs(res["xeb"] - want_xeb) <= 5 * se_xeb


def test_first_mode_gives_one_sample_per_batch(setup):
    n, psi, oq, closed_q, plan, prefixes = setup
    res = sampling.sample(plan, n, oq, closed_q, prefixes, M, np.random.Generator(np.random.PCG64(3003)),
                          mode="first")
    assert 0.95 * len(prefixes) <= res["n_samples"] <= len(prefixes)
    x = res["bitstrings"]
    assert stats.rel_l2(res["amplitudes"].cpu().numpy(), psi[x]) <= 1e-5
