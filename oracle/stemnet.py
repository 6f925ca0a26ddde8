"""Value of a stem network, step by step, in FP64 (paper §A.1-§A.3).

A *stem plan* (plain data) describes a network made of an initial stem
tensor and branch tensors that the stem absorbs one after another:

    {"open_labels":   [...],  # output index, first label most significant
     "sliced_labels": [...],  # summed over; slice id bit (n-1-j) = label j
     "proj_labels":   [...],  # fixed per batch entry, not summed
     "stem":     {"labels": [...], "data": array of shape (2,)*rank},
     "branches": [{"labels": [...], "data": array}, ...]}

For one slice id s and one projected assignment p, every tensor carrying a
sliced or projected label is replaced by its sub-tensor at those values
(§A.1 slicing: each assignment of the sliced edges induces a sub-network).
Then the stem absorbs branch i (i = 1..n): the two tensors are contracted
over every label they share that no later branch carries and that is not
open (§3 Schroedinger method; §A.2 stems and branches).  The final tensor,
transposed to the open-label order, is the slice's value; the sum over all
slices is the value of the unsliced network (§A.1).

Parity pins (tests/test_oracle_stemnet.py): on tiny random stem networks the
per-slice value equals the literal Feynman-path sum of ``network``; the sum
over slices equals the unsliced value; the single-step row formula
``step_rows`` equals ``contract_step`` at every row; a slice of two stems
joined at the root equals the path sum of the whole network.  Plans made from
circuits are pinned against the state vector in the planner tests.
"""

from __future__ import annotations

import numpy as np


def _fix(labels, arr, assign):
    """Sub-tensor with the labels in ``assign`` fixed to their values."""
    idx = []
    keep = []
    for x in labels:
        if x in assign:
            idx.append(int(assign[x]))
        else:
            idx.append(slice(None))
            keep.append(x)
    return tuple(keep), np.asarray(arr)[tuple(idx)]


def slice_assignment(plan: dict, slice_id: int) -> dict:
    sl = list(plan.get("sliced_labels", []))
    n = len(sl)
    return {x: (slice_id >> (n - 1 - j)) & 1 for j, x in enumerate(sl)}


def proj_assignment(plan: dict, proj: int) -> dict:
    pl = list(plan.get("proj_labels", []))
    n = len(pl)
    return {x: (proj >> (n - 1 - j)) & 1 for j, x in enumerate(pl)}


def contract_step(stem, branch, keep):
    """One pairwise contraction: sum over shared labels not in ``keep``.

    Result labels: the stem's labels that are not summed, in the stem's
    order, followed by the branch's labels that the stem does not have, in
    the branch's order.  A shared label in ``keep`` stays once (a common
    index of both factors).
    """
    ls, ts = stem
    lb, tb = branch
    shared = [x for x in ls if x in lb]
    summed = [x for x in shared if x not in keep]
    batch = [x for x in shared if x in keep]
    out = [x for x in ls if x not in summed] + [x for x in lb if x not in ls]
    if batch:
        letters = {}
        for x in list(ls) + list(lb):
            if x not in letters:
                n = len(letters)
                letters[x] = chr(ord("a") + n) if n < 26 else chr(ord("A") + n - 26)
        spec = ("".join(letters[x] for x in ls) + "," + "".join(letters[x] for x in lb)
                + "->" + "".join(letters[x] for x in out))
        return tuple(out), np.einsum(spec, ts, tb)
    ia = [list(ls).index(x) for x in summed]
    ib = [list(lb).index(x) for x in summed]
    res = np.tensordot(np.asarray(ts, dtype=np.complex128),
                       np.asarray(tb, dtype=np.complex128), axes=(ia, ib))
    return tuple(out), res


def run_slice(plan: dict, slice_id: int = 0, proj: int = 0, keep_steps=False):
    """Value of one slice (and one projected assignment) of a stem plan.

    Returns (value, steps): value has shape (2,)*n_open in open-label order;
    steps is a list of (labels, tensor) after each absorbed branch when
    ``keep_steps`` is true, else None.
    """
    assign = slice_assignment(plan, slice_id)
    assign.update(proj_assignment(plan, proj))
    stem = _fix(plan["stem"]["labels"], plan["stem"]["data"], assign)
    stem = (stem[0], np.asarray(stem[1], dtype=np.complex128))
    branches = [_fix(b["labels"], b["data"], assign) for b in plan["branches"]]
    open_set = set(plan.get("open_labels", []))
    later = [set() for _ in branches]
    acc = set()
    for i in range(len(branches) - 1, -1, -1):
        later[i] = set(acc)
        acc.update(branches[i][0])
    steps = [] if keep_steps else None
    for i, br in enumerate(branches):
        stem = contract_step(stem, br, later[i] | open_set)
        if keep_steps:
            steps.append(stem)
    labels, arr = stem
    order = list(plan.get("open_labels", []))
    if sorted(labels) != sorted(order):
        raise ValueError(f"final labels {sorted(labels)} != open labels {sorted(order)}")
    perm = [list(labels).index(x) for x in order]
    return np.transpose(arr, perm), steps


def sliced_sum(plan: dict, slice_ids=None, proj: int = 0) -> np.ndarray:
    """Sum of ``run_slice`` over the given slice ids (default: all)."""
    n_sl = len(plan.get("sliced_labels", []))
    if slice_ids is None:
        slice_ids = range(1 << n_sl)
    total = None
    for s in slice_ids:
        v, _ = run_slice(plan, s, proj)
        total = v.copy() if total is None else total + v
    return total


def unsliced_value(plan: dict, proj: int = 0) -> np.ndarray:
    """Value with the sliced labels treated as ordinary summed labels.

    Contracts the same tensors in the same order, but sliced labels are
    summed inside the steps instead of being enumerated outside.
    """
    assign = proj_assignment(plan, proj)
    stem = _fix(plan["stem"]["labels"], plan["stem"]["data"], assign)
    branches = [_fix(b["labels"], b["data"], assign) for b in plan["branches"]]
    open_set = set(plan.get("open_labels", []))
    later = []
    acc = set()
    for i in range(len(branches) - 1, -1, -1):
        later.append(set(acc))
        acc.update(branches[i][0])
    later.reverse()
    for i, br in enumerate(branches):
        stem = contract_step(stem, br, later[i] | open_set)
    labels, arr = stem
    order = list(plan.get("open_labels", []))
    perm = [list(labels).index(x) for x in order]
    return np.transpose(arr, perm)


def join_slice(left: dict, right: dict, open_labels, slice_id: int = 0, proj: int = 0):
    """One slice of two stems joined at the root (paper §A.2: the root of
    the contraction tree joins two stems).  Both halves list the same
    sliced and projected labels; each half's slice value is taken as by
    ``run_slice`` and the two are contracted over the labels open in both.
    The result is ordered by ``open_labels`` (the labels open in one half).
    """
    vl, _ = run_slice(left, slice_id, proj)
    vr, _ = run_slice(right, slice_id, proj)
    lo, ro = list(left["open_labels"]), list(right["open_labels"])
    shared = [x for x in lo if x in ro]
    res = np.tensordot(vl, vr, axes=([lo.index(x) for x in shared], [ro.index(x) for x in shared]))
    labels = [x for x in lo if x not in shared] + [x for x in ro if x not in shared]
    return transpose_to(labels, res, list(open_labels))


def join_sliced_sum(left: dict, right: dict, open_labels, slice_ids=None, proj: int = 0):
    """Sum of ``join_slice`` over the given slice ids (default: all)."""
    n_sl = len(left.get("sliced_labels", []))
    if slice_ids is None:
        slice_ids = range(1 << n_sl)
    total = None
    for s in slice_ids:
        v = join_slice(left, right, open_labels, s, proj)
        total = v.copy() if total is None else total + v
    return total


def transpose_to(labels, arr, order):
    """Tensor with its axes reordered to ``order`` (a permutation of labels)."""
    perm = [list(labels).index(x) for x in order]
    return np.transpose(np.asarray(arr), perm)


def step_rows(stem_labels, stem_entry, branch_labels, branch_data, out_labels,
              out_index, keep=()):
    """Entries of one contraction step computed one output index at a time.

    ``stem_entry(flat_indices)`` returns stem values (complex) at flat C-order
    indices over ``stem_labels``; the step's output is indexed by
    ``out_labels`` (any order of the result labels).  For each requested flat
    output index the value is the sum over the summed labels' assignments of
    stem[...] * branch[...] (definition of one pairwise contraction, §A.1).
    Used where the full stem is too large to materialise in FP64.
    """
    stem_labels = list(stem_labels)
    branch_labels = list(branch_labels)
    bdata = np.asarray(branch_data, dtype=np.complex128)
    summed = [x for x in stem_labels if x in branch_labels and x not in set(keep)]
    n_sum = len(summed)
    out_labels = list(out_labels)
    n_out = len(out_labels)
    out_index = np.asarray(out_index, dtype=np.int64)
    # bits of every requested output index
    out_bits = {x: (out_index >> (n_out - 1 - j)) & 1 for j, x in enumerate(out_labels)}
    res = np.zeros(out_index.shape, dtype=np.complex128)
    n_s = len(stem_labels)
    for k in range(1 << n_sum):
        kbits = {x: (k >> (n_sum - 1 - j)) & 1 for j, x in enumerate(summed)}
        s_idx = np.zeros(out_index.shape, dtype=np.int64)
        for j, x in enumerate(stem_labels):
            bit = kbits[x] if x in kbits else out_bits[x]
            s_idx += np.asarray(bit, dtype=np.int64) << (n_s - 1 - j)
        b_idx = tuple(np.broadcast_to(kbits[x] if x in kbits else out_bits[x],
                                      out_index.shape) for x in branch_labels)
        res += stem_entry(s_idx) * bdata[b_idx]
    return res
