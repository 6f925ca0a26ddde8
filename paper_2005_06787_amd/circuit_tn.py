"""Circuit to tensor network, on the host, for plan creation (paper §3, §A.1).

The random circuits of paper §2 are plain data (``workloads.circuits``):
moments of named single-qubit gates and of qubit pairs that get fSim.  This
module turns one into a tensor network -- one tensor per gate, a |0> vector
per input wire, and per output wire either an open leg, a <b| vector
(a closed qubit with a known bit) or a projected leg (a closed qubit whose
bit varies over a batch) -- and simplifies it by absorbing every tensor of
rank <= 2 into a neighbour, so single-qubit gates and boundary vectors
disappear into the two-qubit gates.

Gate matrices (paper §2): sqrt(X), sqrt(Y) and sqrt(W), W = (X + Y)/sqrt(2),
are the matrices (I - i G)/sqrt(2) for G in {X, Y, W} -- a rotation by pi/2
about the gate's axis, exp(-i pi/4 G), which squares to -i G; entry by entry
these are the three matrices the paper lists.  fSim(theta,
phi) acts on |01>, |10> as the rotation [[cos, -i sin], [-i sin, cos]] and
puts the phase exp(-i phi) on |11>.
"""

from __future__ import annotations

import itertools
import math

import numpy as np

_PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)


def single_qubit_gate(name: str) -> np.ndarray:
    if name == "id":
        return np.eye(2, dtype=np.complex128)
    axis = {"sqrt_x": _PAULI_X, "sqrt_y": _PAULI_Y,
            "sqrt_w": (_PAULI_X + _PAULI_Y) / math.sqrt(2.0)}.get(name)
    if axis is None:
        raise ValueError(f"unknown gate {name!r}")
    return (np.eye(2) - 1j * axis) / math.sqrt(2.0)


def fsim_gate(theta: float, phi: float) -> np.ndarray:
    """4x4, basis index 2*bit(first qubit) + bit(second qubit)."""
    if theta == math.pi / 2:
        c, s = 0.0, 1.0
    else:
        c, s = math.cos(theta), math.sin(theta)
    g = np.eye(4, dtype=np.complex128)
    g[1:3, 1:3] = [[c, -1j * s], [-1j * s, c]]
    g[3, 3] = np.exp(-1j * phi)
    return g


class Network:
    """Tensors with labels; every label is on one or two tensors."""

    def __init__(self):
        self.tensors: dict[int, tuple[tuple, np.ndarray]] = {}
        self._next_id = itertools.count()
        self.open_labels: list = []
        self.proj_labels: list = []

    def add(self, labels, data) -> int:
        i = next(self._next_id)
        self.tensors[i] = (tuple(labels), np.asarray(data, dtype=np.complex128))
        return i

    def owners(self) -> dict:
        own: dict = {}
        for i, (lab, _) in self.tensors.items():
            for x in lab:
                own.setdefault(x, []).append(i)
        return own


def circuit_network(circuit: dict, open_qubits=(), closed_bits=None, proj_qubits=()) -> Network:
    """Network of <b| U |0^n>: open qubits keep an open leg (in the order of
    ``open_qubits``), projected qubits a dangling leg (order of
    ``proj_qubits``), the others get <closed_bits[q]|."""
    n = circuit["n_qubits"]
    open_qubits = list(open_qubits)
    proj_qubits = list(proj_qubits)
    closed_bits = dict(closed_bits or {})
    net = Network()
    counter = itertools.count()
    wire = [next(counter) for _ in range(n)]
    for q in range(n):
        net.add((wire[q],), [1.0, 0.0])
    g2 = fsim_gate(circuit["theta"], circuit["phi"]).reshape(2, 2, 2, 2)
    for moment in circuit["moments"]:
        if moment["kind"] == "1q":
            for q, name in enumerate(moment["gates"]):
                new = next(counter)
                net.add((new, wire[q]), single_qubit_gate(name))
                wire[q] = new
        else:
            for q1, q2 in moment["pairs"]:
                o1, o2 = next(counter), next(counter)
                net.add((o1, o2, wire[q1], wire[q2]), g2)
                wire[q1], wire[q2] = o1, o2
    for q in range(n):
        if q in open_qubits or q in proj_qubits:
            continue
        bra = np.zeros(2)
        bra[int(closed_bits.get(q, 0))] = 1.0
        net.add((wire[q],), bra)
    net.open_labels = [wire[q] for q in open_qubits]
    net.proj_labels = [wire[q] for q in proj_qubits]
    return net


def contract_two(a, b, keep=()):
    """Contract (labels, data) pairs over their shared labels not in ``keep``;
    shared labels in ``keep`` stay once (diagonal).  Result: a's remaining
    labels, then b's new labels."""
    la, ta = a
    lb, tb = b
    keep = set(keep)
    shared = [x for x in la if x in lb]
    summed = [x for x in shared if x not in keep]
    out = [x for x in la if x not in summed] + [x for x in lb if x not in la]
    letters = {}
    for x in list(la) + list(lb):
        if x not in letters:
            k = len(letters)
            letters[x] = chr(ord("a") + k) if k < 26 else chr(ord("A") + k - 26)
    spec = ("".join(letters[x] for x in la) + "," + "".join(letters[x] for x in lb) + "->"
            + "".join(letters[x] for x in out))
    return tuple(out), np.einsum(spec, ta, tb, optimize=True)


def simplify(net: Network, keep=()) -> Network:
    """Absorb every tensor of rank <= 2 into the neighbour it shares the most
    labels with (ties: the lower-rank neighbour, then the lower id), until
    none is left that has a neighbour.  Labels in ``keep`` (sliced ones) are
    kept as diagonal indices rather than summed."""
    keep = set(keep)
    changed = True
    while changed:
        changed = False
        own = net.owners()
        for i in sorted(net.tensors):
            lab, _ = net.tensors[i]
            if len(lab) > 2:
                continue
            nbrs = {}
            for x in lab:
                for j in own.get(x, []):
                    if j != i and j in net.tensors:
                        nbrs[j] = nbrs.get(j, 0) + 1
            if not nbrs:
                continue
            j = min(nbrs, key=lambda k: (-nbrs[k], len(net.tensors[k][0]), k))
            merged = contract_two(net.tensors[j], net.tensors[i], keep)
            del net.tensors[i]
            net.tensors[j] = merged
            changed = True
            break
    return net
