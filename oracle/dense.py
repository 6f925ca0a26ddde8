"""Plain definitions of the two operations of one stem step.

* ``permute_labels``: a tensor with bond dimension 2 everywhere, stored in C
  order over a label list, re-stored in C order over a permuted label list.
  Equivalently out[pi(a)] = in[a] where pi moves every address bit to the
  position of its label in the new list.  This is the "transposition" that
  pairwise contraction leaves open (§3, §A.1).
* ``cgemm``: complex matrix product C = A B in complex128 (one pairwise
  contraction of §A.1 written as a matrix product once the summed labels
  are the columns of A and the rows of B).

Pins (tests/test_oracle_dense.py): ``permute_labels`` against an explicit
per-entry bit loop; ``cgemm`` against explicit triple sums on small shapes
and against the real 2x2 block embedding [[re, im], [-im, re]].
"""

from __future__ import annotations

import numpy as np


def permute_labels(data, labels_in, labels_out) -> np.ndarray:
    """Re-store a flat 2^r tensor from C order over labels_in to labels_out."""
    r = len(labels_in)
    t = np.asarray(data).reshape((2,) * r)
    perm = [list(labels_in).index(x) for x in labels_out]
    return np.ascontiguousarray(np.transpose(t, perm)).reshape(-1)


def permute_bits_loop(data, labels_in, labels_out) -> np.ndarray:
    """Same as ``permute_labels`` by an explicit loop over entries (tiny)."""
    r = len(labels_in)
    data = np.asarray(data).reshape(-1)
    out = np.empty_like(data)
    pos_out = {x: r - 1 - j for j, x in enumerate(labels_out)}
    for a in range(1 << r):
        b = 0
        for j, x in enumerate(labels_in):
            bit = (a >> (r - 1 - j)) & 1
            b |= bit << pos_out[x]
        out[b] = data[a]
    return out


def cgemm(a, b) -> np.ndarray:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return a @ b
