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
