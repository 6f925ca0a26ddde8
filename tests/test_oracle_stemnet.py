"""Pins of the stem-network oracle against the literal Feynman-path sum."""
import numpy as np
import pytest

from oracle import network as tn
from oracle import stemnet


def _rand(rng, rank):
    return rng.standard_normal((2,) * rank) + 1j * rng.standard_normal((2,) * rank)


def random_stem_plan(seed, n_steps=4, stem_rank=4, n_sliced=2, n_proj=1):
    """A small stem network: each label in two tensors, or one if dangling."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nxt = stem_rank
    stem_labels = list(range(stem_rank))
    cur = list(stem_labels)
    branches = []
    dangling = []
    for i in range(n_steps):
        s = int(rng.integers(1, min(3, len(cur)) + 1))
        shared = [cur[int(p)] for p in rng.choice(len(cur), size=s, replace=False)]
        f = int(rng.integers(0, 3))
        f = max(f, s + 2 - len(cur))  # keep the stem at rank >= 2
        new = list(range(nxt, nxt + f))
        nxt += f
        # a dangling label: appears in this branch only
        if rng.random() < 0.5:
            dangling.append(nxt)
            new_d = [nxt]
            nxt += 1
        else:
            new_d = []
        lab = shared + new + new_d
        order = rng.permutation(len(lab))
        lab = [lab[int(o)] for o in order]
        branches.append({"labels": lab, "data": _rand(rng, len(lab))})
        cur = [x for x in cur if x not in shared] + new
    open_labels = list(cur)
    rng.shuffle(open_labels)
    internal = [x for x in range(nxt) if x not in set(open_labels) and x not in set(dangling)]
    sliced = [internal[int(p)] for p in rng.choice(len(internal), size=min(n_sliced, len(internal)), replace=False)]
    proj = dangling[:n_proj]
    # any other dangling label becomes open too
    open_labels += [x for x in dangling[n_proj:]]
    return {
        "open_labels": [int(x) for x in open_labels],
        "sliced_labels": [int(x) for x in sliced],
        "proj_labels": [int(x) for x in proj],
        "stem": {"labels": stem_labels, "data": _rand(rng, stem_rank)},
        "branches": branches,
    }


def _all_tensors(plan):
    return [(tuple(plan["stem"]["labels"]), plan["stem"]["data"])] + \
        [(tuple(b["labels"]), b["data"]) for b in plan["branches"]]


def _fixed_network(plan, assign):
    out = []
    for lab, arr in _all_tensors(plan):
        idx = tuple(int(assign[x]) if x in assign else slice(None) for x in lab)
        out.append((tuple(x for x in lab if x not in assign), arr[idx]))
    return out


@pytest.mark.parametrize("seed", range(8))
def test_slice_value_equals_bruteforce(seed):
    plan = random_stem_plan(seed)
    n_sl = len(plan["sliced_labels"])
    n_pr = len(plan["proj_labels"])
    for p in range(1 << n_pr):
        for s in range(1 << n_sl):
            assign = stemnet.slice_assignment(plan, s)
            assign.update(stemnet.proj_assignment(plan, p))
            ref = tn.value_bruteforce(_fixed_network(plan, assign), plan["open_labels"])
            got, steps = stemnet.run_slice(plan, s, p, keep_steps=True)
            assert np.allclose(got, ref, atol=1e-10)
            assert len(steps) == len(plan["branches"])


@pytest.mark.parametrize("seed", range(8))
def test_sliced_sum_equals_unsliced(seed):
    plan = random_stem_plan(seed + 100)
    n_pr = len(plan["proj_labels"])
    for p in range(1 << n_pr):
        assign = stemnet.proj_assignment(plan, p)
        ref = tn.value_bruteforce(_fixed_network(plan, assign), plan["open_labels"])
        assert np.allclose(stemnet.sliced_sum(plan, proj=p), ref, atol=1e-10)
        assert np.allclose(stemnet.unsliced_value(plan, proj=p), ref, atol=1e-10)


def test_slice_bit_order_msb_first():
    plan = {"sliced_labels": [7, 3, 5]}
    assert stemnet.slice_assignment(plan, 0b100) == {7: 1, 3: 0, 5: 0}
    assert stemnet.slice_assignment(plan, 0b011) == {7: 0, 3: 1, 5: 1}


@pytest.mark.parametrize("seed", range(4))
def test_step_rows_equals_contract_step(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    sl = [0, 1, 2, 3, 4, 5, 6]
    stem = _rand(rng, len(sl))
    shared = [5, 1, 3]
    bl = shared + [10, 11]
    br = _rand(rng, len(bl))
    lab, full = stemnet.contract_step((tuple(sl), stem), (tuple(bl), br), keep=set())
    order = [11, 0, 2, 10, 4, 6]
    ref = stemnet.transpose_to(lab, full, order).reshape(-1)
    flat = stem.reshape(-1)
    idx = rng.choice(ref.size, size=20, replace=False)
    got = stemnet.step_rows(sl, lambda i: flat[i], bl, br, order, idx)
    assert np.allclose(got, ref[idx], atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_hyperedge_slices_equal_bruteforce(seed):
    """Networks where a step keeps labels it shares with the stem (a later
    branch or the result carries them again): the stem oracle keeps them
    as common indices and still equals the literal path sum."""
    from workloads.networks import random_stem_network

    plan = random_stem_network(300 + seed, stem_rank=5, n_steps=5, s_range=(1, 3),
                               f_range=(0, 2), n_sliced=1, n_proj=1, batch_prob=0.6,
                               rank_bounds=(2, 7), dtype=np.complex128)
    counts = {}
    for lab, _ in _all_tensors(plan):
        for x in lab:
            counts[x] = counts.get(x, 0) + 1
    opened = set(plan["open_labels"])
    assert any(c >= 3 for c in counts.values()) or any(
        counts[x] >= 2 for x in opened), "no hyperedge drawn"
    for p in range(1 << len(plan["proj_labels"])):
        for s in range(1 << len(plan["sliced_labels"])):
            assign = stemnet.slice_assignment(plan, s)
            assign.update(stemnet.proj_assignment(plan, p))
            ref = tn.value_bruteforce(_fixed_network(plan, assign), plan["open_labels"])
            got, _ = stemnet.run_slice(plan, s, p)
            assert np.allclose(got, ref, atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2, 7, 8, 9])
def test_join_slice_equals_bruteforce(seed):
    """Two stems joined at the root (paper §A.2): cutting a network into a
    left stem (stem and first branches) and a right stem (the other
    branches), and contracting their slice values over the shared labels,
    gives the path sum of the whole network at every slice and projected
    assignment, whatever the cut."""
    from workloads.networks import random_stem_network, split_stem_network

    plan = random_stem_network(400 + seed, stem_rank=5, n_steps=5, s_range=(1, 3),
                               f_range=(0, 2), n_sliced=2, n_proj=1, rank_bounds=(2, 7),
                               batch_prob=0.4, n_open_final=3, dtype=np.complex128)
    cuts = 0
    for h in range(1, len(plan["branches"])):
        try:
            left, right = split_stem_network(plan, h)
        except ValueError:
            continue
        cuts += 1
        for p in range(1 << len(plan["proj_labels"])):
            for s in range(1 << len(plan["sliced_labels"])):
                assign = stemnet.slice_assignment(plan, s)
                assign.update(stemnet.proj_assignment(plan, p))
                ref = tn.value_bruteforce(_fixed_network(plan, assign), plan["open_labels"])
                got = stemnet.join_slice(left, right, plan["open_labels"], s, p)
                assert np.allclose(got, ref, atol=1e-10), (h, s, p)
        total = stemnet.join_sliced_sum(left, right, plan["open_labels"])
        assert np.allclose(total, stemnet.sliced_sum(plan), atol=1e-10)
    assert cuts >= 1


def test_join_of_two_vectors_is_their_inner_product():
    """Special case written out: two rank-3 stems without branches sharing
    labels 1 and 2, joined over them, are the matrix sum over x1, x2 of
    l[x0, x1, x2] r[x2, x1, x5], ordered (x5, x0)."""
    rng = np.random.Generator(np.random.PCG64(7))
    lv = _rand(rng, 3)
    rv = _rand(rng, 3)
    left = {"open_labels": [0, 1, 2], "sliced_labels": [], "proj_labels": [],
            "stem": {"labels": [0, 1, 2], "data": lv}, "branches": []}
    right = {"open_labels": [2, 1, 5], "sliced_labels": [], "proj_labels": [],
             "stem": {"labels": [2, 1, 5], "data": rv}, "branches": []}
    got = stemnet.join_slice(left, right, [5, 0])
    ref = np.zeros((2, 2), dtype=np.complex128)
    for x5 in range(2):
        for x0 in range(2):
            ref[x5, x0] = sum(lv[x0, x1, x2] * rv[x2, x1, x5] for x1 in range(2) for x2 in range(2))
    assert np.allclose(got, ref, atol=1e-13)
