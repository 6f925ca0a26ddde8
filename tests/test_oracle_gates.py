"""Pins of the gate matrices against closed forms of paper §2."""
import cmath
import math

import numpy as np
import pytest

from oracle.gates import fsim, gate_1q

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
W = (X + Y) / math.sqrt(2.0)


@pytest.mark.parametrize("name", ["sqrt_x", "sqrt_y", "sqrt_w", "id"])
def test_unitary(name):
    u = gate_1q(name)
    assert np.allclose(u.conj().T @ u, np.eye(2), atol=1e-15)


def test_fsim_unitary():
    for th, ph in [(math.pi / 2, math.pi / 6), (0.3, 1.1)]:
        u = fsim(th, ph)
        assert np.allclose(u.conj().T @ u, np.eye(4), atol=1e-15)


@pytest.mark.parametrize("name,target", [("sqrt_x", X), ("sqrt_y", Y), ("sqrt_w", W)])
def test_square_roots(name, target):
    # each gate squared is the named Pauli-type operator times -i
    u = gate_1q(name)
    assert np.allclose(u @ u, -1j * target, atol=1e-15)


def test_sqrt_x_on_zero():
    v = gate_1q("sqrt_x") @ np.array([1, 0], dtype=complex)
    assert np.allclose(v, np.array([1, -1j]) / math.sqrt(2.0), atol=1e-15)


def test_fsim_closed_forms():
    u = fsim(math.pi / 2, math.pi / 6)
    e01 = np.zeros(4, complex); e01[1] = 1
    e11 = np.zeros(4, complex); e11[3] = 1
    e10 = np.zeros(4, complex); e10[2] = 1
    assert np.array_equal(u @ e01, -1j * e10)
    assert np.allclose(u @ e11, cmath.exp(-1j * math.pi / 6) * e11, atol=1e-15)
    # theta = pi/2 uses exact cos = 0 and sin = 1
    assert u[1, 1] == 0 and u[2, 2] == 0


def test_unknown_gate():
    with pytest.raises(ValueError):
        gate_1q("t")
