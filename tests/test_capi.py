"""Host-side checks of libstemgpu: it loads, exports every declared symbol,
and its host planner computes the step shapes of paper §A.1 (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2005_06787_amd import _capi as C
from paper_2005_06787_amd import stem_plan_validate
from workloads.networks import random_stem_network

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "stemgpu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stem_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    handle = ctypes.CDLL(C.LIB_PATH)
    for name in names:
        assert hasattr(handle, name), name
    # and the binding declares a signature for each of them
    assert set(names) <= set(C.SIGNATURES)


def _expected_steps(net):
    """Step shapes recomputed from the label lists (paper §A.1 step cost)."""
    fixed = set(net["sliced_labels"]) | set(net["proj_labels"])
    cur = [x for x in net["stem"]["labels"] if x not in fixed]
    peak = len(cur)
    out = []
    for b in net["branches"]:
        lab = [x for x in b["labels"] if x not in fixed]
        shared = [x for x in cur if x in lab]
        free = [x for x in lab if x not in cur]
        s, f = len(shared), len(free)
        out.append((len(cur) - s, s, f))
        cur = [x for x in cur if x not in shared] + free
        peak = max(peak, len(cur))
    return out, peak


@pytest.mark.parametrize("seed", range(10))
def test_validate_step_shapes(seed):
    net = random_stem_network(seed, stem_rank=9, n_steps=7, n_open_final=5)
    summ = stem_plan_validate(net)
    steps, peak = _expected_steps(net)
    assert summ["n_steps"] == len(steps)
    assert summ["peak_rank"] == peak
    assert summ["n_slices"] == 1 << len(net["sliced_labels"])
    flops = sum(8.0 * 2 ** (m + s + f) for m, s, f in steps)
    nbytes = sum(8.0 * (2 ** (m + s) + 2 ** (m + f) + 2 ** (s + f)) for m, s, f in steps)
    assert summ["flops_per_slice"] == flops
    assert summ["bytes_per_slice"] == nbytes


def _tiny():
    rng = np.random.Generator(np.random.PCG64(0))
    d = lambda r: rng.standard_normal((2,) * r) + 0j  # noqa: E731
    return {"open_labels": [3], "sliced_labels": [], "proj_labels": [],
            "stem": {"labels": [0, 1], "data": d(2)},
            "branches": [{"labels": [1, 2], "data": d(2)},
                         {"labels": [0, 2, 3], "data": d(3)}]}


def test_validate_accepts_tiny():
    s = stem_plan_validate(_tiny())
    assert s["n_steps"] == 2 and s["n_open"] == 1


def test_error_codes():
    net = _tiny()
    bad = dict(net, open_labels=[2])            # 2 joins two tensors, 3 dangles
    with pytest.raises(C.StemError) as e:
        stem_plan_validate(bad)
    assert e.value.status == C.STEM_ELABEL
    bad = dict(net, branches=[{"labels": [1, 5], "data": np.ones((2, 2))}] + net["branches"])
    with pytest.raises(C.StemError) as e:       # label 5 in one tensor, not open
        stem_plan_validate(bad)
    assert e.value.status == C.STEM_ELABEL
    with pytest.raises(C.StemError) as e:
        stem_plan_validate(net, max_rank=1)     # stem of rank 2
    assert e.value.status == C.STEM_ESHAPE
    bad = dict(net, sliced_labels=[3])          # open and sliced at once
    with pytest.raises(C.StemError) as e:
        stem_plan_validate(bad)
    assert e.value.status == C.STEM_ELABEL
    assert C.lib().stem_plan_validate(None, None) == C.STEM_EINVAL
    assert b"null" in C.lib().stem_last_error()


def test_null_handles_are_refused_on_the_host():
    """Entry points that take a plan or join handle refuse null before any
    device work (no GPU needed)."""
    lib = C.lib()
    h = ctypes.c_void_p()
    n = ctypes.c_uint64()
    assert lib.stem_step_sched_set(None, 0, 1, 1, 4096, -1, 0) == C.STEM_EINVAL
    assert lib.stem_join_create(None, None, 0, None, ctypes.byref(h)) == C.STEM_EINVAL
    assert h.value is None
    assert lib.stem_join_create(None, None, 0, None, None) == C.STEM_EINVAL
    assert lib.stem_join_workspace_bytes(None, 1, ctypes.byref(n)) == C.STEM_EINVAL
    assert lib.stem_join_contract(None, 0, 1, None, 1, None, 0, None, 0, None) == C.STEM_EINVAL
    assert lib.stem_join_destroy(None) == C.STEM_OK


def test_sliced_label_in_no_tensor_is_accepted():
    """A sliced or projected label need not occur in the plan's tensors (the
    two halves of a join list the same ones); the step shapes are unchanged."""
    net = _tiny()
    base = stem_plan_validate(net)
    more = dict(net, sliced_labels=list(net.get("sliced_labels", [])) + [99],
                proj_labels=list(net.get("proj_labels", [])) + [98])
    s = stem_plan_validate(more)
    assert s["n_slices"] == 2 * base["n_slices"]
    assert s["flops_per_slice"] == base["flops_per_slice"]


def test_hyperedge_steps_are_batched():
    """Label 1 joins three tensors: step 0 keeps it (a batched product over
    its 2 values), step 2 sums it."""
    from paper_2005_06787_amd import runtime_model as rm

    net = _tiny()
    hyper = dict(net, branches=net["branches"] + [{"labels": [1], "data": np.ones(2)}])
    s = stem_plan_validate(hyper)
    assert s["n_steps"] == 3
    steps = rm.plan_steps(hyper)
    assert [st.n_batch for st in steps] == [1, 0, 0]
    # step 0: stem [0, 1] x branch [1, 2], 1 kept: M = 2 (label 0), K = 1, N = 2
    assert (steps[0].M, steps[0].K, steps[0].N) == (2, 1, 2)
    assert steps[0].flops == 8.0 * 2 * (2 * 1 * 2)


def test_too_many_batch_labels_in_one_step():
    rng = np.random.Generator(np.random.PCG64(1))
    d = lambda r: rng.standard_normal((2,) * r) + 0j  # noqa: E731
    # the stem and branch 0 share 0..4, all needed again by branch 1
    net = {"open_labels": [5], "sliced_labels": [], "proj_labels": [],
           "stem": {"labels": [0, 1, 2, 3, 4], "data": d(5)},
           "branches": [{"labels": [0, 1, 2, 3, 4, 5], "data": d(6)},
                        {"labels": [0, 1, 2, 3, 4], "data": d(5)}]}
    with pytest.raises(C.StemError) as e:
        stem_plan_validate(net)
    assert e.value.status == C.STEM_EUNSUPPORTED


def test_status_strings():
    for s in range(8):
        assert C.lib().stem_status_str(s)
