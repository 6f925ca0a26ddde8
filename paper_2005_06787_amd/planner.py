"""Stem planner: circuit -> sliced stem network (host side, not timed).

Plan creation is preprocessing; the paper excludes it from its runtimes
(§A.4) and pre-computes the branches on the host (§A.3).  The paper finds
the stem with hypergraph partitioning and local search (§4, §A.2); this
planner is a simpler stand-in that produces the same kind of object, a
slicing scheme (E_s, T) whose tree T is a stem (§A.1, §A.2):

1. Build the circuit's network and absorb rank <= 2 tensors (circuit_tn).
2. Linear stem order: start from a random tensor and repeatedly absorb the
   neighbouring tensor that leaves the smallest stem (ties: the one sharing
   the most labels; then random), over many seeded trials.  A trial is
   scored after step 3 by (peak width, time complexity tc).
3. Greedy slicing (§4, §A.2 dynamic slicing): add the label, among those on
   the widest stems, whose removal gives the smallest tc (ties: lowest
   label), until the width target or the sliced-label count is met.
   tc((E_s, T)) = 2^|E_s| * sum over steps of 2^|E_step \\ E_s| (§A.1).
   Optionally the best order is sliced again with stem-focused local
   optimisation after every pick (§A.2: every window of consecutive
   tensors takes its best order).
4. The first tensors of the order are pre-contracted into the initial stem
   while its rank stays small; the rest are grouped into branches of
   consecutive tensors (§A.3, branch merging), up to a branch rank limit.
   The merge points minimise the summed step time of a cost model (a
   roofline of the rates the kernels sustain, or the learned model), by
   dynamic programming over the order.
5. Branches and the initial stem are contracted on the host in FP64 and
   stored as complex64 (§A.3: computed once, shared by all slices).
"""

from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np

from .circuit_tn import circuit_network, contract_two, simplify

# Roofline model of one step on one MI355X (used to decide branch merges).
HBM_BYTES_PER_S = 5.0e12      # sustained stream rate, below the 8 TB/s peak
MFMA_FP32_FLOPS = 1.0e14      # sustained FP32 MFMA rate, below the 157 TF peak
LAUNCH_S = 4.0e-6             # per kernel launch


def step_time(r_in: int, s: int, f: int, permuted: bool = False) -> float:
    """Modelled seconds of one stem step: stem rank r_in, s summed, f new."""
    m = 2.0 ** (r_in - s)
    k, n = 2.0 ** s, 2.0 ** f
    t_mem = 8.0 * (m * k + m * n + k * n) / HBM_BYTES_PER_S
    t_flop = 8.0 * m * k * n / MFMA_FP32_FLOPS
    t = max(t_mem, t_flop) + LAUNCH_S
    if permuted:
        t += 16.0 * m * k / HBM_BYTES_PER_S + LAUNCH_S
    return t


class _Order:
    """A linear order with per-step label sets, for fast slicing updates."""

    def __init__(self, tlabels, order):
        self.order = list(order)
        stems, unions = [], []
        stem = set(tlabels[order[0]])
        stems.append(frozenset(stem))
        for j in order[1:]:
            t = tlabels[j]
            unions.append(frozenset(stem | t))
            stem = stem ^ t
            stems.append(frozenset(stem))
        self.stems = stems        # stem after absorbing order[0..k]
        self.unions = unions      # labels of step k (stem before + tensor)
        # the same sets as 0/1 matrices over the sorted labels
        self.labels = sorted(set().union(*stems, *unions))
        col = {x: i for i, x in enumerate(self.labels)}
        self.smat = np.zeros((len(stems), len(self.labels)), dtype=np.int64)
        self.umat = np.zeros((len(unions), len(self.labels)), dtype=np.int64)
        for k, st in enumerate(stems):
            self.smat[k, [col[x] for x in st]] = 1
        for k, u in enumerate(unions):
            self.umat[k, [col[x] for x in u]] = 1
        self.col = col

    def widths(self, sliced=frozenset()):
        return [len(s - sliced) for s in self.stems]

    def tc(self, sliced=frozenset()):
        return (2.0 ** len(sliced)) * sum(2.0 ** len(u - sliced) for u in self.unions)


def _linear_order(tlabels, owners, rng, noise=0.5):
    n = len(tlabels)
    start = int(rng.integers(n))
    stem = set(tlabels[start])
    order = [start]
    remaining = set(range(n))
    remaining.discard(start)
    while remaining:
        cands = set()
        for x in stem:
            for j in owners.get(x, ()):
                if j in remaining:
                    cands.add(j)
        if not cands:
            cands = remaining
        best, best_key = None, None
        for j in cands:
            t = tlabels[j]
            key = (len(stem ^ t) + noise * rng.random(), -len(stem & t))
            if best_key is None or key < best_key:
                best, best_key = j, key
        stem ^= tlabels[best]
        order.append(best)
        remaining.discard(best)
    return order


def greedy_slice(od: _Order, n_sliced=None, max_width=None, forbid=(), rng=None, top: int = 3,
                 start=()):
    """Greedy slicing of a linear order (§4, §A.2 dynamic slicing).

    Each pick adds, among the labels of the widest stems, the one whose
    removal gives the smallest (peak width, tc); ties go to the lowest
    label.  With ``rng`` the pick is uniform among the ``top`` best (the
    randomised variant that draws candidate slicing sets).  All candidates
    of a pick are scored at once: with w_k the width of stem k and u_k the
    size of step k's label set (both without the sliced labels), slicing
    label x gives peak max_k (w_k - [x in stem k]) and
    tc = 2 tc - 2^|E_s| sum_{k: x in step k} 2^u_k (§A.1).
    """
    sliced = []
    fb = np.zeros(len(od.labels), dtype=bool)
    for x in forbid:
        if x in od.col:
            fb[od.col[x]] = True
    taken = np.zeros(len(od.labels), dtype=bool)
    w = od.smat.sum(axis=1)
    u = od.umat.sum(axis=1)
    for x in start:               # labels already sliced
        i = od.col[x]
        taken[i] = True
        sliced.append(x)
        w = w - od.smat[:, i]
        u = u - od.umat[:, i]
    while True:
        peak = int(w.max())
        if n_sliced is not None and len(sliced) >= n_sliced:
            break
        if n_sliced is None and (max_width is None or peak <= max_width):
            break
        cand = od.smat[w == peak].any(axis=0) & ~taken & ~fb
        idx = np.nonzero(cand)[0]
        if not len(idx):
            break
        new_peak = (w[:, None] - od.smat[:, idx]).max(axis=0)
        pw = np.exp2(u.astype(np.float64))
        tc_now = (2.0 ** len(sliced)) * pw.sum()
        new_tc = 2.0 * tc_now - (2.0 ** len(sliced)) * (pw @ od.umat[:, idx])
        keys = sorted(zip(new_peak.tolist(), new_tc.tolist(), [od.labels[i] for i in idx], idx))
        pick = keys[0] if rng is None else keys[int(rng.integers(min(top, len(keys))))]
        i = pick[3]
        taken[i] = True
        sliced.append(od.labels[i])
        w = w - od.smat[:, i]
        u = u - od.umat[:, i]
    return sorted(sliced)


def _label_masks(tlabels):
    bit = {x: 1 << i for i, x in enumerate(sorted(set().union(*tlabels)))}
    return [sum(bit[x] for x in t) for t in tlabels], bit


def local_optimize(tlabels, order, sliced=(), window: int = 4, passes: int = 3):
    """Stem-focused local optimisation (§A.2): slide a window of
    ``window`` consecutive tensors along the order and put them in the
    order (of all window! orders) that gives the least (peak width of the
    whole order, time inside the window); the stems before and after a
    window do not depend on the order within it.  Widths and times leave
    out the sliced labels.
    Repeats until a pass changes nothing (at most ``passes`` passes)."""
    import itertools

    masks, bit = _label_masks(tlabels)
    slm = 0
    for x in sliced:
        slm |= bit.get(x, 0)
    keep = ~slm
    order = list(order)
    n = len(order)
    w = min(window, n - 1)
    if w < 2:
        return order
    for _ in range(passes):
        changed = False
        stems = [masks[order[0]]]
        for j in order[1:]:
            stems.append(stems[-1] ^ masks[j])
        widths = [(st & keep).bit_count() for st in stems]
        suffix = widths[:] + [0]          # suffix[k] = max width of stems k..n-1
        for k in range(n - 1, -1, -1):
            suffix[k] = max(widths[k], suffix[k + 1])
        prefix = 0                        # max width of stems 0..i-1 (as reordered)
        for i in range(1, n - w + 1):
            prefix = max(prefix, (stems[i - 1] & keep).bit_count())
            outside = max(prefix, suffix[i + w] if i + w <= n else 0)
            before = stems[i - 1]
            win = tuple(order[i:i + w])
            best_key, best = None, win
            for perm in itertools.permutations(win):
                st, pk, tc = before, 0, 0.0
                for j in perm:
                    tc += 2.0 ** ((st | masks[j]) & keep).bit_count()
                    st ^= masks[j]
                    pk = max(pk, (st & keep).bit_count())
                key = (max(pk, outside), tc)
                if best_key is None or key < best_key:
                    best_key, best = key, perm
            if best != win:
                order[i:i + w] = list(best)
                st = before
                for k in range(i, i + w):
                    st ^= masks[order[k]]
                    stems[k] = st
                changed = True
        if not changed:
            break
    return order


def refine_scheme(tlabels, order, n_sliced=None, max_width=None, forbid=(), window: int = 4):
    """Dynamic slicing interleaved with local optimisation (§A.2): after
    every greedy pick the order is locally re-optimised for the labels
    sliced so far.  Returns (order, sliced, peak, tc)."""
    order = local_optimize(tlabels, order, (), window)
    sliced = []
    while True:
        od = _Order(tlabels, order)
        peak = max(od.widths(frozenset(sliced)))
        if n_sliced is not None and len(sliced) >= n_sliced:
            break
        if n_sliced is None and (max_width is None or peak <= max_width):
            break
        nxt = greedy_slice(od, n_sliced=len(sliced) + 1, forbid=forbid, start=sliced)
        if len(nxt) == len(sliced):
            break
        sliced = nxt
        order = local_optimize(tlabels, order, sliced, window)
    od = _Order(tlabels, order)
    fs = frozenset(sliced)
    return order, sorted(sliced), max(od.widths(fs)), od.tc(fs)


def find_scheme(tlabels, trials: int, seed: int, n_sliced=None, max_width=None, forbid=(),
                local_window: int = 0):
    """Best linear order + slicing over seeded trials: (order, sliced, peak, tc).

    With ``local_window`` >= 2 the best trial's order is then sliced again
    with local optimisation after every pick (``refine_scheme``), and the
    refined scheme is kept when its (peak width, tc) is lower."""
    owners: dict = {}
    for i, lab in enumerate(tlabels):
        for x in lab:
            owners.setdefault(x, []).append(i)
    rng = np.random.Generator(np.random.PCG64(seed))
    best = None
    for _ in range(trials):
        order = _linear_order(tlabels, owners, rng)
        od = _Order(tlabels, order)
        sl = greedy_slice(od, n_sliced=n_sliced, max_width=max_width, forbid=forbid)
        fs = frozenset(sl)
        key = (max(od.widths(fs)), od.tc(fs))
        if best is None or key < best[0]:
            best = (key, order, sl)
    (peak, tc), order, sl = best
    if local_window >= 2:
        r = refine_scheme(tlabels, order, n_sliced=n_sliced, max_width=max_width, forbid=forbid,
                          window=local_window)
        if (r[2], r[3]) < (peak, tc):
            return r
    return order, sl, peak, tc


def candidate_orders(tlabels, n: int, seed: int, n_sliced=None, max_width=None, forbid=()):
    """n (order, sliced labels) schemes from seeded trials of the linear
    stem search, each order sliced greedily: candidate stem orders."""
    owners: dict = {}
    for i, lab in enumerate(tlabels):
        for x in lab:
            owners.setdefault(x, []).append(i)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        order = _linear_order(tlabels, owners, rng)
        sl = greedy_slice(_Order(tlabels, order), n_sliced=n_sliced, max_width=max_width,
                          forbid=forbid)
        out.append((order, sl))
    return out


def candidate_slicings(tlabels, order, n: int, seed: int, n_sliced=None, max_width=None,
                       forbid=(), top: int = 3):
    """n slicing sets of one order from the randomised greedy slicer
    (distinct sets only, in the order drawn)."""
    od = _Order(tlabels, order)
    rng = np.random.Generator(np.random.PCG64(seed))
    out, seen = [], set()
    for _ in range(n):
        sl = tuple(greedy_slice(od, n_sliced=n_sliced, max_width=max_width, forbid=forbid,
                                rng=rng, top=top))
        if sl not in seen:
            seen.add(sl)
            out.append(list(sl))
    return out


def _group_labels(tlabels, group):
    acc = set()
    for j in group:
        acc ^= tlabels[j]
    return acc


def group_branches(tlabels, order, n_init: int, fixed: set, max_branch_rank: int = 12,
                   merge=True, step_cost=None):
    """Split order[n_init:] into consecutive groups (merged branches).

    Without ``step_cost``: greedy, a tensor joins the current group while
    one merged product is modelled no slower than two (``step_time``).
    With ``step_cost(r_in, s, f) -> seconds``: the partition that minimises
    the summed cost, by dynamic programming over the order (the stem
    before a group does not depend on how earlier tensors were grouped, so
    the optimum over prefixes composes); groups end within
    ``max_branch_rank`` unfixed labels and never pass through more than 4
    labels above it while the host contracts them in order.
    """
    if step_cost is not None and merge:
        return _group_branches_dp(tlabels, order, n_init, fixed, max_branch_rank, step_cost)
    merge = bool(merge)
    stem = _group_labels(tlabels, order[:n_init]) - fixed
    groups = []
    cur = []
    cur_lab = set()

    def cost(st, lab):
        s = len(st & lab)
        f = len(lab - st)
        return step_time(len(st), s, f)

    for j in order[n_init:]:
        t = tlabels[j] - fixed
        if not cur:
            cur, cur_lab = [j], set(t)
            continue
        merged = cur_lab ^ t
        ok = merge and len(merged) <= max_branch_rank
        if ok:
            after_cur = stem ^ cur_lab
            t_sep = cost(stem, cur_lab) + cost(after_cur, t)
            t_merged = cost(stem, merged)
            ok = t_merged <= t_sep
        if ok:
            cur.append(j)
            cur_lab = merged
        else:
            groups.append(cur)
            stem = stem ^ cur_lab
            cur, cur_lab = [j], set(t)
    if cur:
        groups.append(cur)
    return groups


def _group_branches_dp(tlabels, order, n_init, fixed, max_branch_rank, step_cost):
    seq = list(order[n_init:])
    n = len(seq)
    labs = [frozenset(tlabels[j] - fixed) for j in seq]
    stems = [frozenset(_group_labels(tlabels, order[:n_init]) - fixed)]
    for t in labs:
        stems.append(stems[-1] ^ t)
    best = [0.0] + [math.inf] * n
    back = [0] * (n + 1)
    for i in range(n):
        if best[i] == math.inf:
            continue
        st = stems[i]
        g = set()
        for j in range(i, n):
            g ^= labs[j]
            if j > i and len(g) > max_branch_rank:
                if len(g) > max_branch_rank + 4:   # the host contracts groups in order
                    break
                continue
            c = best[i] + step_cost(len(st), len(st & g), len(g - st))
            if c < best[j + 1]:
                best[j + 1], back[j + 1] = c, i
    groups = []
    j = n
    while j > 0:
        i = back[j]
        groups.append(seq[i:j])
        j = i
    return groups[::-1]


def roofline_step_cost(hbm_bytes_per_s: float = 5.0e12, flops_per_s: float = 1.2e14,
                       launch_s: float = 4e-6, slices_in_flight: int = 128):
    """step_cost(r_in, s, f) of one slice on a roofline: max(bytes / bandwidth,
    flops / rate) plus the launch shared by the slices in flight.  The
    defaults are the rates the product kernels sustain on one MI355X in
    FP32 (streaming 5 TB/s, 120 TFLOP/s on MFMA-bound shapes)."""
    def cost(r_in, s, f):
        m, k, n = 2.0 ** (r_in - s), 2.0 ** s, 2.0 ** f
        return (max(8.0 * (m * k + m * n + k * n) / hbm_bytes_per_s,
                    8.0 * m * k * n / flops_per_s) + launch_s / slices_in_flight)
    return cost


def _contract_group(tensors, group, keep):
    acc = tensors[group[0]]
    for j in group[1:]:
        acc = contract_two(acc, tensors[j], keep)
    return acc


def _group_label_list(tensors, group, keep):
    """Labels (in order) of _contract_group's result, without the data."""
    out = list(tensors[group[0]][0])
    for j in group[1:]:
        lb = tensors[j][0]
        summed = {x for x in out if x in lb and x not in keep}
        out = [x for x in out if x not in summed] + [x for x in lb if x not in out]
    return out


class CircuitProblem:
    """A circuit's simplified network and the label sets the planner orders
    (projected labels excluded; open labels may not be sliced)."""

    def __init__(self, circuit: dict, open_qubits=(), closed_bits=None, proj_qubits=()):
        self.net = simplify(circuit_network(circuit, open_qubits, closed_bits, proj_qubits))
        ids = sorted(self.net.tensors)
        self.tensors = [self.net.tensors[i] for i in ids]
        self.proj = set(self.net.proj_labels)
        self.tlabels = [frozenset(x for x in lab if x not in self.proj)
                        for lab, _ in self.tensors]
        self.forbid = set(self.net.open_labels)


def scheme_network(pb: CircuitProblem, order, sliced, *, init_rank: int = 12,
                   max_branch_rank: int = 14, merge: str = "dp", with_data: bool = True,
                   stats: dict | None = None, step_cost=None) -> dict:
    """The stem network of a scheme (order, sliced labels) of a problem.

    Branch merging (§A.3): ``merge`` "dp" picks the merge points that
    minimise the summed ``step_cost`` (default: ``roofline_step_cost()``;
    the MLP's predictions through ``runtime_model.mlp_step_cost``), "greedy"
    merges while the built-in roofline says one larger product is no
    slower than two, "none" keeps one branch per tensor.

    Without data the tensors carry their labels only (for ranking schemes
    by their step shapes); with data the initial stem and the branches are
    contracted on the host in FP64 and stored as complex64.
    """
    tlabels = pb.tlabels
    fixed = set(sliced) | pb.proj
    # initial stem: absorb while the (unfixed) rank stays within init_rank
    n_init = 1
    stem_lab = set(tlabels[order[0]]) - fixed
    while n_init < len(order):
        nxt = stem_lab ^ (tlabels[order[n_init]] - fixed)
        if len(nxt) > init_rank:
            break
        stem_lab = nxt
        n_init += 1
    if merge == "dp":
        groups = group_branches(tlabels, order, n_init, fixed, max_branch_rank, True,
                                step_cost or roofline_step_cost())
    else:
        groups = group_branches(tlabels, order, n_init, fixed, max_branch_rank,
                                merge == "greedy")
    keep = set(sliced)
    if with_data:
        stem = _contract_group(pb.tensors, order[:n_init], keep)
        stem_d = {"labels": [int(x) for x in stem[0]], "data": stem[1].astype(np.complex64)}
    else:
        stem_d = {"labels": [int(x) for x in _group_label_list(pb.tensors, order[:n_init], keep)]}
    branches = []
    for g in groups:
        if with_data:
            lab, data = _contract_group(pb.tensors, g, keep)
            branches.append({"labels": [int(x) for x in lab], "data": data.astype(np.complex64)})
        else:
            branches.append({"labels": [int(x) for x in _group_label_list(pb.tensors, g, keep)]})
    st = dict(stats or {})
    st.update({"n_tensors": len(pb.tensors), "n_branches": len(branches), "n_init": n_init})
    return {
        "open_labels": [int(x) for x in pb.net.open_labels],
        "sliced_labels": [int(x) for x in sorted(sliced)],
        "proj_labels": [int(x) for x in pb.net.proj_labels],
        "stem": stem_d,
        "branches": branches,
        "stats": st,
    }


class _SideProblem:
    """The tensors of one side of a two-sided scheme, as a problem of its
    own whose open labels are the side's open labels and its cut labels."""

    def __init__(self, pb: CircuitProblem, idx, open_labels):
        self.tensors = [pb.tensors[i] for i in idx]
        self.tlabels = [pb.tlabels[i] for i in idx]
        self.proj = pb.proj
        self.forbid = set(open_labels)
        self.net = SimpleNamespace(open_labels=list(open_labels),
                                   proj_labels=list(pb.net.proj_labels))


def two_sided_networks(pb: CircuitProblem, order, sliced, h: int, **kw):
    """Two stems meeting at the root (paper §A.2, a root in the middle of
    the stem): the left stem grows from order[0] through order[h-1], the
    right stem from the last tensor of the order back to order[h].  Each
    side keeps open the network's open labels it carries and the unsliced
    labels between the sides (the cut); the join contracts the two final
    stems over the cut.  Every cut of the order is the same edge set seen
    from either side, so each side's stem widths are the one-sided stem's
    widths on its part of the order.

    Returns (left network, right network, join open labels); ``kw`` goes to
    ``scheme_network`` for both sides.
    """
    n = len(order)
    if not 1 <= h < n:
        raise ValueError("cut outside [1, len(order))")
    left_idx = [int(i) for i in order[:h]]
    right_idx = [int(i) for i in reversed(order[h:])]
    fixed = set(sliced) | pb.proj
    lab_l = _group_labels(pb.tlabels, left_idx) - fixed
    lab_r = _group_labels(pb.tlabels, right_idx) - fixed
    cut = sorted(lab_l & lab_r)
    opened = [int(x) for x in pb.net.open_labels]
    l_open = [x for x in opened if x in lab_l] + cut
    r_open = [x for x in opened if x in lab_r] + cut
    left = scheme_network(_SideProblem(pb, left_idx, l_open), list(range(len(left_idx))),
                          sliced, **kw)
    right = scheme_network(_SideProblem(pb, right_idx, r_open), list(range(len(right_idx))),
                           sliced, **kw)
    return left, right, opened


def plan_circuit(circuit: dict, open_qubits=(), closed_bits=None, proj_qubits=(), *,
                 n_sliced=None, max_width=None, trials: int = 64, seed: int = 0,
                 init_rank: int = 12, max_branch_rank: int = 14, merge: str = "dp",
                 step_cost=None, local_window: int = 0) -> dict:
    """Sliced stem network of a circuit's amplitudes.

    ``open_qubits`` stay open (result index, first qubit most significant),
    ``proj_qubits`` are fixed per batch entry (projected assignment bits in
    the same order), the other qubits are closed with ``closed_bits``.
    Returns the network dictionary plus a "stats" entry.
    """
    pb = CircuitProblem(circuit, open_qubits, closed_bits, proj_qubits)
    order, sliced, peak, tc = find_scheme(pb.tlabels, trials, seed, n_sliced=n_sliced,
                                          max_width=max_width, forbid=pb.forbid,
                                          local_window=local_window)
    stats = {"peak_width": int(peak), "tc": float(tc),
             "log2_tc": float(math.log2(tc)) if tc > 0 else 0.0, "order": list(order)}
    return scheme_network(pb, order, sliced, init_rank=init_rank,
                          max_branch_rank=max_branch_rank, merge=merge, stats=stats,
                          step_cost=step_cost)
