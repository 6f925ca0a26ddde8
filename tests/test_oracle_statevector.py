"""Pins of the FP64 state-vector oracle."""
import cmath
import math

import numpy as np

from oracle import statevector as sv
from oracle import stats
from workloads import circuits


def _circ(n, moments, theta=math.pi / 2, phi=math.pi / 6):
    return {"n_qubits": n, "theta": theta, "phi": phi, "moments": moments}


def test_one_qubit_hand_worked():
    psi = sv.run(_circ(1, [{"kind": "1q", "gates": ["sqrt_x"]}]))
    assert np.allclose(psi, np.array([1, -1j]) / math.sqrt(2), atol=1e-15)
    psi = sv.run(_circ(1, [{"kind": "1q", "gates": ["sqrt_y"]}]))
    assert np.allclose(psi, np.array([1, 1]) / math.sqrt(2), atol=1e-15)


def test_qubit_zero_is_most_significant_bit():
    # sqrt(X) on qubit 0 of two: amplitude of x=0b10 (qubit 0 set) is -i/sqrt2
    psi = sv.run(_circ(2, [{"kind": "1q", "gates": ["sqrt_x", "id"]}]))
    assert np.allclose(psi, np.array([1, 0, -1j, 0]) / math.sqrt(2), atol=1e-15)


def test_fsim_on_basis_states():
    # |01> -> -i|10>, built by X on qubit 1 (sqrt_x twice = -iX)
    prep = [{"kind": "1q", "gates": ["id", "sqrt_x"]}, {"kind": "1q", "gates": ["id", "sqrt_x"]}]
    psi = sv.run(_circ(2, prep + [{"kind": "2q", "pairs": [[0, 1]]}]))
    # state before fSim is -i|01>; after it (-i)(-i)|10> = -|10>
    assert np.allclose(psi, np.array([0, 0, -1, 0]), atol=1e-15)
    prep2 = prep + [{"kind": "1q", "gates": ["sqrt_x", "id"]}, {"kind": "1q", "gates": ["sqrt_x", "id"]}]
    psi = sv.run(_circ(2, prep2 + [{"kind": "2q", "pairs": [[0, 1]]}]))
    # before: (-i)^2 |11> = -|11>; fSim multiplies |11> by exp(-i pi/6)
    assert np.allclose(psi, np.array([0, 0, 0, -cmath.exp(-1j * math.pi / 6)]), atol=1e-15)


def test_norm_is_one():
    c = circuits.make_circuit(3, 4, 6, seed=3)
    psi = sv.run(c)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12


def test_batch_amplitudes_matches_direct_indexing():
    c = circuits.make_circuit(2, 3, 4, seed=4)
    psi = sv.run(c)
    open_q = [4, 1]
    closed = [0, 2, 3, 5]
    bits = [1, 0, 1, 1]
    got = sv.batch_amplitudes(psi, 6, open_q, closed, bits)
    for a in range(4):
        full = {4: (a >> 1) & 1, 1: a & 1}
        full.update(dict(zip(closed, bits)))
        x = sum(full[q] << (5 - q) for q in range(6))
        assert got[a] == psi[x]


def test_porter_thomas_on_20_qubits():
    # 4x5 grid, 8 cycles: the output distribution is close to Porter-Thomas
    c = circuits.make_circuit(4, 5, 8, seed=1)
    psi = sv.run(c)
    p = np.abs(psi) ** 2
    assert abs(p.sum() - 1.0) < 1e-12
    assert stats.porter_thomas_ks(p, 1 << 20) < 0.02
    assert 0.75 < stats.collision_xeb(psi, 20) < 1.25
    # bitstrings sampled from the ideal distribution give XEB near 1,
    # uniform bitstrings give XEB near 0
    rng = np.random.Generator(np.random.PCG64(2001))
    xs = rng.choice(1 << 20, size=4096, p=p / p.sum())
    assert 0.75 < stats.xeb(psi[xs], 20) < 1.25
    ys = rng.integers(0, 1 << 20, size=4096)
    assert abs(stats.xeb(psi[ys], 20)) < 0.15
