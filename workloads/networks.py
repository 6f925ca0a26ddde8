"""Seeded random stem networks (structure and values only; no contraction).

A stem network is the plain dictionary both sides read:

    {"open_labels": [...], "sliced_labels": [...], "proj_labels": [...],
     "stem": {"labels": [...], "data": complex array of shape (2,)*rank},
     "branches": [{"labels": [...], "data": complex array}, ...]}

Every label joins exactly two tensors, except open labels (one tensor),
projected labels (a dangling leg of one tensor, fixed per batch entry),
sliced labels (any joining label, enumerated outside the contraction) and,
with ``batch_prob`` > 0, hyperedges: a label a step shares with the stem
and keeps, so that a later step or the result carries it again.
"""

from __future__ import annotations

import numpy as np


def _cgauss(rng, shape, scale):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * (scale / np.sqrt(2.0))


def random_stem_network(seed: int, stem_rank: int = 8, n_steps: int = 6, *,
                        s_range=(1, 4), f_range=(0, 4), rank_bounds=None,
                        n_sliced: int = 2, n_proj: int = 1, n_open_final: int | None = None,
                        fastest_prob: float = 0.3, batch_prob: float = 0.0,
                        dtype=np.complex64) -> dict:
    """Draw a random stem network.

    At each step the branch shares s labels with the stem (s uniform in
    s_range; with probability ``fastest_prob`` the s fastest stem labels,
    else a uniform subset) in a random order, and adds f new labels.  Ranks
    stay within ``rank_bounds`` (default [1, stem_rank + 4]).  Branch
    entries are complex Gaussian with variance 1/2^s so the stem's magnitude
    stays roughly constant.  A projected label is a dangling leg added to a
    random tensor; sliced labels are drawn among the joining labels.  If
    ``n_open_final`` is given, closing steps (f = 0) bring the final rank to
    at most that value.  With ``batch_prob`` > 0 each shared label of a step
    (at most 2 per step) is kept in the stem with that probability instead
    of being summed: a hyperedge joining the stem, this branch and a later
    branch or the result.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = rank_bounds if rank_bounds is not None else (1, stem_rank + 4)
    nxt = stem_rank
    stem_labels = [int(x) for x in rng.permutation(stem_rank)]
    cur = list(stem_labels)
    joins = []
    branches = []

    def add_step(s, f):
        nonlocal nxt, cur
        if rng.random() < fastest_prob:
            shared = cur[len(cur) - s:]
        else:
            shared = [cur[int(p)] for p in sorted(rng.choice(len(cur), size=s, replace=False))]
        kept = []
        if batch_prob > 0:
            for x in shared:
                if len(kept) < 2 and rng.random() < batch_prob:
                    kept.append(x)
        new = list(range(nxt, nxt + f))
        nxt += f
        lab = shared + new
        order = rng.permutation(len(lab))
        lab = [lab[int(o)] for o in order]
        n_sum = len(shared) - len(kept)
        data = _cgauss(rng, (2,) * len(lab), 1.0 / np.sqrt(2.0 ** n_sum))
        branches.append({"labels": lab, "data": data})
        joins.extend(x for x in shared if x not in kept)
        gone = set(shared) - set(kept)
        cur = [x for x in cur if x not in gone] + new

    for _ in range(n_steps):
        R = len(cur)
        for _try in range(100):
            s = int(rng.integers(s_range[0], s_range[1] + 1))
            f = int(rng.integers(f_range[0], f_range[1] + 1))
            if 0 <= s <= R and lo <= R - s + f <= hi:
                break
        else:
            s, f = min(1, R), 1
        add_step(s, f)
    if n_open_final is not None:
        while len(cur) > n_open_final:
            s = min(len(cur) - n_open_final, int(rng.integers(1, 7)))
            add_step(s, 0)
    open_labels = list(cur)
    rng.shuffle(open_labels)
    # projected labels: dangling legs on random tensors (stem or a branch)
    tensors = [("stem", None)] + [("branch", i) for i in range(len(branches))]
    stem_data = _cgauss(rng, (2,) * stem_rank, 1.0)
    proj = []
    for _ in range(n_proj):
        kind, i = tensors[int(rng.integers(0, len(tensors)))]
        lab = nxt
        nxt += 1
        proj.append(lab)
        vec = _cgauss(rng, (2,), 1.0)
        if kind == "stem":
            pos = int(rng.integers(0, len(stem_labels) + 1))
            stem_labels.insert(pos, lab)
            stem_data = np.moveaxis(np.multiply.outer(stem_data, vec), -1, pos)
        else:
            b = branches[i]
            pos = int(rng.integers(0, len(b["labels"]) + 1))
            b["labels"].insert(pos, lab)
            b["data"] = np.moveaxis(np.multiply.outer(b["data"], vec), -1, pos)
    sliced = []
    if n_sliced and joins:
        picks = rng.choice(len(joins), size=min(n_sliced, len(joins)), replace=False)
        sliced = [int(joins[int(p)]) for p in picks]
    for b in branches:
        b["data"] = np.ascontiguousarray(b["data"]).astype(dtype)
    return {
        "open_labels": [int(x) for x in open_labels],
        "sliced_labels": sliced,
        "proj_labels": proj,
        "stem": {"labels": [int(x) for x in stem_labels],
                 "data": np.ascontiguousarray(stem_data).astype(dtype)},
        "branches": branches,
    }


def split_stem_network(net: dict, h: int) -> tuple[dict, dict]:
    """Cut a stem network into two stems that meet at the root (structure
    only): the left one is the stem and branches [0, h), the right one has
    branch h as its initial stem and branches (h, n) after it.  Each half
    keeps open the labels it shares with the other half and the network's
    open labels it carries; both list the network's sliced and projected
    labels.  The labels open in exactly one half are the network's open
    labels, which is checked: an open label carried by both halves (a
    hyperedge at the root) raises ValueError.
    """
    br = net["branches"]
    if not 1 <= h < len(br):
        raise ValueError("split point outside [1, n_branches)")
    fixed = set(net["sliced_labels"]) | set(net["proj_labels"])
    opened = set(net["open_labels"])
    left_t = [net["stem"]] + br[:h]
    right_t = br[h:]

    def labels_of(ts):
        seen = []
        for t in ts:
            for x in t["labels"]:
                if x not in seen:
                    seen.append(int(x))
        return seen

    ll, rl = labels_of(left_t), labels_of(right_t)
    if any(x in opened and x in rl for x in ll):
        raise ValueError("an open label is carried by both halves")
    l_open = [x for x in ll if x not in fixed and (x in opened or x in rl)]
    r_open = [x for x in rl if x not in fixed and (x in opened or x in ll)]
    common = {"sliced_labels": list(net["sliced_labels"]), "proj_labels": list(net["proj_labels"])}
    left = dict(common, open_labels=l_open, stem=net["stem"], branches=list(br[:h]))
    right = dict(common, open_labels=r_open, stem=br[h], branches=list(br[h + 1:]))
    return left, right
