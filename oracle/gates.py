"""Gate matrices of the random circuit family (paper §2), in complex128.

sqrt(X), sqrt(Y), sqrt(W) and fSim(theta, phi) are written out from their
definitions in §2 ("id", the identity, is accepted for hand-built test
circuits; the generator never emits it).  sqrt(i) and sqrt(-i) are the principal roots
exp(+i pi/4) and exp(-i pi/4).  For theta = pi/2 the cosine and sine are
taken as exactly 0 and 1.

Pins (tests/test_oracle_gates.py): unitarity; sqrt(G)^2 equals X, Y and
W = (X + Y)/sqrt(2) up to a global phase; fSim(pi/2, phi) on |01> gives
-i|10> and on |11> gives exp(-i phi)|11>.
"""

from __future__ import annotations

import math

import numpy as np

_R2 = 1.0 / math.sqrt(2.0)


def gate_1q(name: str) -> np.ndarray:
    """2x2 matrix of a named single-qubit gate (rows = output index)."""
    if name == "id":
        return np.eye(2, dtype=np.complex128)
    if name == "sqrt_x":
        return _R2 * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)
    if name == "sqrt_y":
        return _R2 * np.array([[1, -1], [1, 1]], dtype=np.complex128)
    if name == "sqrt_w":
        sqrt_i = complex(math.cos(math.pi / 4), math.sin(math.pi / 4))
        sqrt_mi = complex(math.cos(math.pi / 4), -math.sin(math.pi / 4))
        return _R2 * np.array([[1, -sqrt_i], [sqrt_mi, 1]], dtype=np.complex128)
    raise ValueError(f"unknown single-qubit gate {name!r}")


def fsim(theta: float, phi: float) -> np.ndarray:
    """4x4 fSim(theta, phi); basis index = 2*bit(first qubit) + bit(second)."""
    if theta == math.pi / 2:
        c, s = 0.0, 1.0
    else:
        c, s = math.cos(theta), math.sin(theta)
    u = np.zeros((4, 4), dtype=np.complex128)
    u[0, 0] = 1.0
    u[1, 1] = c
    u[1, 2] = -1j * s
    u[2, 1] = -1j * s
    u[2, 2] = c
    u[3, 3] = complex(math.cos(phi), -math.sin(phi))
    return u
