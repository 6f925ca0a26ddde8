"""Host logic of frugal rejection sampling (no GPU): acceptance, the
first accepted candidate in a visiting order, and bitstring assembly."""
import numpy as np

from paper_2005_06787_amd import sampling


def test_accept_threshold():
    n = 3                                     # N = 8
    p = np.array([[0.5, 0.05, 0.0, 0.125]])   # N p = 4, 0.4, 0, 1
    u = np.array([[0.99, 0.39, 0.0, 0.5]])
    acc = sampling.accept(p, n, 2.0, u)       # thresholds 1, 0.2, 0, 0.5
    assert acc.tolist() == [[True, False, False, False]]


def test_first_accepted_follows_order():
    acc = np.array([[False, True, True, False], [False, False, False, False]])
    order = np.array([[2, 1, 0, 3], [0, 1, 2, 3]])
    assert sampling.first_accepted(acc, order).tolist() == [2, -1]


def test_bitstrings_place_prefix_and_open_bits():
    # 5 qubits: open (4, 1), projected (0, 3), qubit 2 absent from both (0)
    x = sampling.bitstrings([4, 1], [0, 3], 5, np.array([0b10, 0b01]), np.array([0b01, 0b10]))
    # prefix 10 -> q0 = 1, q3 = 0; open 01 -> q4 = 0, q1 = 1  => 1 1 0 0 0
    # prefix 01 -> q0 = 0, q3 = 1; open 10 -> q4 = 1, q1 = 0  => 0 0 0 1 1
    assert x.tolist() == [0b11000, 0b00011]
