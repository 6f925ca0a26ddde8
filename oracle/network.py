"""A circuit as a tensor network and the network's value (paper §3, §A.1).

A network is a list of (labels, array) pairs plus a list of open labels.
Every bond has dimension 2 (§A.1).  The value T_H[b] is the sum, over all
assignments of the labels that agree with b on the open labels, of the
product of the tensors' entries (the Feynman-path sum of §A.1).

Two independent ways to compute it:

* ``value_bruteforce`` -- the literal sum over every assignment of every
  label (tiny networks only).
* ``value_pairwise``   -- repeated pairwise contraction (the Schroedinger
  method of §3): pick two tensors, contract them over the labels that occur
  in no other tensor and are not open, replace them by the result.  §A.1
  states the value does not depend on the order; the order policy is
  "random" (seeded) or "greedy" (smallest result first).

Circuit to network: |0> on each wire, one rank-2 tensor U[out, in] per
single-qubit gate, one rank-4 tensor U[o1, o2, i1, i2] per fSim, and at the
end either an open label (open qubit) or a rank-1 <b| (closed qubit).

Pins (tests/test_oracle_network.py): brute force equals the state vector on
every bitstring of tiny grids; pairwise contraction in several random orders
equals the brute force and the state vector; a hand-built network with
known value.
"""

from __future__ import annotations

import itertools

import numpy as np

from .gates import fsim, gate_1q


def circuit_network(circuit: dict, open_qubits=(), closed_bits=None):
    """Tensor network of <b_closed| U |0^n> with the open qubits left open.

    ``closed_bits``: dict qubit -> bit for every qubit not in ``open_qubits``
    (default all zero).  Returns (tensors, open_labels) with open labels in
    the order of ``open_qubits``.
    """
    n = circuit["n_qubits"]
    open_qubits = list(open_qubits)
    closed_bits = dict(closed_bits or {})
    counter = itertools.count()
    wire = [next(counter) for _ in range(n)]
    tensors = []
    for q in range(n):
        tensors.append(((wire[q],), np.array([1.0, 0.0], dtype=np.complex128)))
    u2 = fsim(circuit["theta"], circuit["phi"]).reshape(2, 2, 2, 2)
    for moment in circuit["moments"]:
        if moment["kind"] == "1q":
            for q, name in enumerate(moment["gates"]):
                new = next(counter)
                tensors.append(((new, wire[q]), gate_1q(name)))
                wire[q] = new
        else:
            for q1, q2 in moment["pairs"]:
                o1, o2 = next(counter), next(counter)
                tensors.append(((o1, o2, wire[q1], wire[q2]), u2.copy()))
                wire[q1], wire[q2] = o1, o2
    for q in range(n):
        if q in open_qubits:
            continue
        b = int(closed_bits.get(q, 0))
        bra = np.zeros(2, dtype=np.complex128)
        bra[b] = 1.0
        tensors.append(((wire[q],), bra))
    open_labels = [wire[q] for q in open_qubits]
    return tensors, open_labels


def all_labels(tensors):
    labels = []
    seen = set()
    for lab, _ in tensors:
        for x in lab:
            if x not in seen:
                seen.add(x)
                labels.append(x)
    return labels


def value_bruteforce(tensors, open_labels) -> np.ndarray:
    """Literal Feynman-path sum of §A.1 over every assignment (tiny only).

    Returns the value with shape (2,)*len(open_labels), open labels in order.
    """
    labels = all_labels(tensors)
    for x in open_labels:
        if x not in labels:
            raise ValueError(f"open label {x} is in no tensor")
    closed = [x for x in labels if x not in set(open_labels)]
    if len(labels) > 22:
        raise ValueError("network too large for the brute-force sum")
    pos = {x: i for i, x in enumerate(closed + list(open_labels))}
    n_closed = len(closed)
    n_all = len(pos)
    # every assignment of every label, as rows of bits
    grid = ((np.arange(1 << n_all)[:, None] >> np.arange(n_all - 1, -1, -1)[None, :])
            & 1).astype(np.uint8)
    prod = np.ones(1 << n_all, dtype=np.complex128)
    for lab, arr in tensors:
        idx = tuple(grid[:, pos[x]] for x in lab)
        prod *= arr[idx]
    # rows are ordered with the closed labels most significant: summing over
    # the closed block leaves the open assignment as the row index
    out = prod.reshape(1 << n_closed, 1 << (n_all - n_closed)).sum(axis=0)
    return out.reshape((2,) * len(open_labels))


def contract_pair(a, b, keep):
    """Contract two (labels, array) tensors over shared labels not in ``keep``.

    Shared labels in ``keep`` (needed by another tensor, or open) stay in the
    result as a common index.  Result labels: a's kept labels, then b's
    labels that a does not have.
    """
    la, ta = a
    lb, tb = b
    shared = [x for x in la if x in lb]
    summed = [x for x in shared if x not in keep]
    batch = [x for x in shared if x in keep]
    out = [x for x in la if x not in summed] + [x for x in lb if x not in la]
    if not batch:
        ia = [la.index(x) for x in summed]
        ib = [lb.index(x) for x in summed]
        res = np.tensordot(ta, tb, axes=(ia, ib))
        res_labels = [x for x in la if x not in summed] + [x for x in lb if x not in summed]
        perm = [res_labels.index(x) for x in out]
        return tuple(out), np.transpose(res, perm)
    letters = {}
    for x in list(la) + list(lb):
        if x not in letters:
            letters[x] = chr(ord("a") + len(letters)) if len(letters) < 26 else \
                chr(ord("A") + len(letters) - 26)
    spec = "".join(letters[x] for x in la) + "," + "".join(letters[x] for x in lb) + \
        "->" + "".join(letters[x] for x in out)
    return tuple(out), np.einsum(spec, ta, tb)


def value_pairwise(tensors, open_labels, order="greedy", seed=0,
                   max_rank=None) -> np.ndarray:
    """Network value by repeated pairwise contraction (§3).

    order="random": a uniformly random pair of tensors sharing a label.
    order="greedy": the sharing pair whose result has the fewest labels
    (ties: lowest positions in the current list).  Disconnected tensors are
    combined by outer product at the end.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    work = [(tuple(lab), np.asarray(arr)) for lab, arr in tensors]
    open_set = set(open_labels)
    while len(work) > 1:
        count = {}
        for lab, _ in work:
            for x in lab:
                count[x] = count.get(x, 0) + 1
        pairs = []
        for i in range(len(work)):
            si = set(work[i][0])
            for j in range(i + 1, len(work)):
                if si & set(work[j][0]):
                    pairs.append((i, j))
        if not pairs:
            pairs = [(0, 1)]
        if order == "random":
            i, j = pairs[int(rng.integers(0, len(pairs)))]
        elif order == "greedy":
            best = None
            for i, j in pairs:
                li, lj = set(work[i][0]), set(work[j][0])
                shared = li & lj
                gone = {x for x in shared if count[x] == 2 and x not in open_set}
                rank = len(li | lj) - len(gone)
                key = (rank, i, j)
                if best is None or key < best:
                    best = key
            _, i, j = best
        else:
            raise ValueError(order)
        a, b = work[i], work[j]
        keep = set(open_set)
        for k, (lab, _) in enumerate(work):
            if k not in (i, j):
                keep.update(lab)
        res = contract_pair(a, b, keep)
        if max_rank is not None and len(res[0]) > max_rank:
            raise MemoryError(f"pairwise contraction reached rank {len(res[0])}")
        work = [t for k, t in enumerate(work) if k not in (i, j)] + [res]
    lab, arr = work[0]
    # scalars left over from closed sub-networks were folded in above; any
    # open label must now be present
    perm = [lab.index(x) for x in open_labels]
    return np.transpose(arr, perm)
