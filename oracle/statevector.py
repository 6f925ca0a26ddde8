"""FP64 state-vector simulation of a circuit (paper §2 semantics).

psi starts as |0...0>; each gate is applied with ``tensordot`` on its qubit
axes.  Qubit 0 is the most significant bit of a bitstring integer x, so the
amplitude <x|U|0^n> is psi.reshape(-1)[x].

Pins (tests/test_oracle_statevector.py): hand-worked one- and two-qubit
cases; norm 1 to 1e-12; agreement with the literal Feynman-path sum of
``network`` on tiny grids and with pairwise contraction on larger ones;
Porter-Thomas statistics on 20 qubits.
"""

from __future__ import annotations

import numpy as np

from .gates import fsim, gate_1q


def apply_1q(psi: np.ndarray, u: np.ndarray, q: int) -> np.ndarray:
    out = np.tensordot(u, psi, axes=([1], [q]))
    return np.moveaxis(out, 0, q)


def apply_2q(psi: np.ndarray, u4: np.ndarray, q1: int, q2: int) -> np.ndarray:
    u = u4.reshape(2, 2, 2, 2)
    out = np.tensordot(u, psi, axes=([2, 3], [q1, q2]))
    return np.moveaxis(out, [0, 1], [q1, q2])


def run(circuit: dict) -> np.ndarray:
    """Final state as a flat complex128 vector of length 2^n."""
    n = circuit["n_qubits"]
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    u2 = fsim(circuit["theta"], circuit["phi"])
    for moment in circuit["moments"]:
        if moment["kind"] == "1q":
            for q, name in enumerate(moment["gates"]):
                psi = apply_1q(psi, gate_1q(name), q)
        else:
            for q1, q2 in moment["pairs"]:
                psi = apply_2q(psi, u2, q1, q2)
    return np.ascontiguousarray(psi).reshape(-1)


def amplitudes(psi: np.ndarray, bitstrings) -> np.ndarray:
    return psi[np.asarray(list(bitstrings), dtype=np.int64)]


def batch_amplitudes(psi: np.ndarray, n_qubits: int, open_qubits, closed_qubits,
                     closed_bits) -> np.ndarray:
    """The 2^len(open) amplitudes with closed qubits fixed (paper §3 batch).

    Output index: open qubits in the given order, first one most significant.
    """
    t = psi.reshape((2,) * n_qubits)
    idx = [slice(None)] * n_qubits
    for q, b in zip(closed_qubits, closed_bits):
        idx[q] = int(b)
    sub = t[tuple(idx)]
    # remaining axes are the open qubits in ascending order
    remaining = sorted(open_qubits)
    perm = [remaining.index(q) for q in open_qubits]
    return np.ascontiguousarray(np.transpose(sub, perm)).reshape(-1)
