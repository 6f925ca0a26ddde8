"""Time complexity and contraction width of a contraction scheme (§A.1).

For one pairwise step of tensors A and B, E_AB is the set of labels on A or
B and E*_AB the labels of E_AB that are open or carried by another tensor;
the step costs 2^|E_AB| (multiply-adds) in time and 2^|E*_AB| in space.
tc(T) sums the step times, cw(T) is the largest |E*|, and with a sliced set
E_s, tc((E_s, T)) = 2^|E_s| tc(T) with the sliced labels removed from the
network first (§A.1, slicing).

One multiply-add of complex numbers is 8 real floating-point operations;
this is the convention under which Table 1's FLOPS efficiencies and the
closing estimate of §A.4 come out of the printed costs and times.

Pins (tests/test_oracle_cost.py): a matrix chain with hand-computed cost;
step times equal M*K*N of the matrix product form; Table 1's efficiencies
and the §A.4 runtime estimate from the printed numbers.
"""

from __future__ import annotations


def scheme_cost(leaves, steps, open_labels=(), sliced=()):
    """Cost of contracting ``leaves`` (label sets) along ``steps``.

    ``steps`` is a list of (i, j) pairs of indices into the current list of
    tensors; the result is appended at the end and i, j are removed.
    Returns (tc, cw, per_step) with per_step a list of (|E|, |E*|).
    Sliced labels are deleted from every tensor first and tc is multiplied
    by 2^|sliced|.
    """
    sliced = set(sliced)
    work = [frozenset(x for x in lab if x not in sliced) for lab in leaves]
    open_set = set(open_labels) - sliced
    per_step = []
    for i, j in steps:
        a, b = work[i], work[j]
        others = set()
        for k, lab in enumerate(work):
            if k not in (i, j):
                others |= lab
        e = a | b
        e_star = frozenset(x for x in e if x in others or x in open_set)
        per_step.append((len(e), len(e_star)))
        work = [lab for k, lab in enumerate(work) if k not in (i, j)] + [e_star]
    tc = sum(2 ** e for e, _ in per_step) * (2 ** len(sliced))
    cw = max((s for _, s in per_step), default=0)
    return tc, cw, per_step


def stem_scheme_steps(n_branches: int):
    """Steps of a stem that absorbs branches 1..n in order (stem is leaf 0)."""
    steps = []
    # after each step the stem result sits at the end of the list; branch i
    # keeps index 0 because the earlier branches have been removed
    for i in range(n_branches):
        cur = n_branches - i  # position of the running stem
        steps.append((cur if i else 0, 0 if i else 1))
    return steps


def flops(tc_macs: float) -> float:
    """Real floating-point operations of tc complex multiply-adds."""
    return 8.0 * tc_macs
