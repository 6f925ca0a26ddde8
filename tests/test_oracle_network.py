"""Pins of the tensor-network value: brute force vs state vector vs pairwise."""
import math

import numpy as np
import pytest

from oracle import network as tn
from oracle import statevector as sv
from workloads import circuits


@pytest.mark.parametrize("rows,cols,cycles", [(2, 2, 1), (2, 2, 2), (1, 3, 2), (2, 3, 1)])
def test_bruteforce_equals_statevector_all_open(rows, cols, cycles):
    c = circuits.make_circuit(rows, cols, cycles, seed=rows * 10 + cols + cycles)
    n = c["n_qubits"]
    tensors, open_labels = tn.circuit_network(c, open_qubits=range(n))
    got = tn.value_bruteforce(tensors, open_labels).reshape(-1)
    psi = sv.run(c)
    assert np.allclose(got, psi, atol=1e-12)


def test_bruteforce_closed_amplitude():
    c = circuits.make_circuit(2, 2, 2, seed=9)
    psi = sv.run(c)
    for x in [0, 5, 9, 15]:
        bits = {q: (x >> (3 - q)) & 1 for q in range(4)}
        tensors, open_labels = tn.circuit_network(c, open_qubits=[], closed_bits=bits)
        got = tn.value_bruteforce(tensors, open_labels)
        assert abs(complex(got) - psi[x]) < 1e-12


@pytest.mark.parametrize("rows,cols,cycles", [(2, 3, 4), (3, 3, 8), (3, 3, 5)])
def test_pairwise_random_orders_equal_statevector(rows, cols, cycles):
    c = circuits.make_circuit(rows, cols, cycles, seed=rows + cols * cycles)
    n = c["n_qubits"]
    psi = sv.run(c)
    tensors, open_labels = tn.circuit_network(c, open_qubits=range(n))
    for seed in range(3):
        got = tn.value_pairwise(tensors, open_labels, order="random", seed=seed)
        assert np.allclose(got.reshape(-1), psi, atol=1e-12)
    got = tn.value_pairwise(tensors, open_labels, order="greedy")
    assert np.allclose(got.reshape(-1), psi, atol=1e-12)


def test_pairwise_partial_open_equals_statevector_batch():
    c = circuits.make_circuit(3, 3, 6, seed=21)
    psi = sv.run(c)
    open_q = [2, 5, 1]
    closed = [q for q in range(9) if q not in open_q]
    bits = [1, 0, 0, 1, 1, 0]
    tensors, open_labels = tn.circuit_network(c, open_q, dict(zip(closed, bits)))
    got = tn.value_pairwise(tensors, open_labels, order="greedy").reshape(-1)
    ref = sv.batch_amplitudes(psi, 9, open_q, closed, bits)
    assert np.allclose(got, ref, atol=1e-12)


def test_hand_built_trace():
    # value of A(a,b) B(b,a) with no open labels is trace(A B)
    a = np.array([[1, 2j], [3, 4]], dtype=complex)
    b = np.array([[5, 6], [7j, 8]], dtype=complex)
    expect = (1 * 5 + 2j * 7j) + (3 * 6 + 4 * 8)
    tensors = [((0, 1), a), ((1, 0), b)]
    assert abs(complex(tn.value_bruteforce(tensors, [])) - expect) < 1e-12
    assert abs(complex(tn.value_pairwise(tensors, [])) - expect) < 1e-12


def test_hand_built_open_vector():
    # v(a) = sum_b M[a,b] w[b]
    m = np.array([[1, 2], [3, 4j]], dtype=complex)
    w = np.array([1j, -1], dtype=complex)
    tensors = [((0, 1), m), ((1,), w)]
    expect = np.array([1j - 2, 3j - 4j])
    assert np.allclose(tn.value_bruteforce(tensors, [0]), expect)
    assert np.allclose(tn.value_pairwise(tensors, [0]), expect)
