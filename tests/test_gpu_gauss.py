"""The 3M FP32 product (three real products per complex one) against the
FP64 oracle.

Random stem networks whose steps have whole 3M tiles (K a multiple of 8,
N of 16, M of 64) run with every such step forced to the 3M kernel in
several launch schedules (row blocks per wave, column tiles, workgroups,
branch fragments in LDS or not, 4- or 8-wave workgroups); every slice matches the oracle at
relative L2 <= 1e-5 and the real-embedding result closely, also on
batched steps of hyperedge networks.  Forcing the 3M product where it
does not apply is refused.
"""
import numpy as np
import pytest

from oracle import stats, stemnet
from workloads.networks import random_stem_network

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import Plan  # noqa: E402
from paper_2005_06787_amd import _capi as C  # noqa: E402

NETS = [
    # (seed, stem_rank, n_steps, s_range, f_range, n_sliced, n_proj, n_open_final)
    (51, 14, 6, (3, 5), (4, 6), 2, 1, 6),
    (52, 18, 6, (3, 7), (4, 6), 1, 0, 8),     # K up to 128, several chunks and tiles
    (53, 12, 8, (3, 4), (4, 5), 2, 1, None),
]
SCHEDULES = [(1, 1, 1024, -1), (1, 4, 4096, 1), (2, 2, 16384, 0), (4, 1, 4096, -1),
             (1, 4, 4096, 2), (2, 2, 1024, 2), (1, 4, 4096, 3)]


def _net(cfg):
    seed, r, n, sr, fr, nsl, npr, nof = cfg
    return random_stem_network(seed, stem_rank=r, n_steps=n, s_range=sr, f_range=fr,
                               n_sliced=nsl, n_proj=npr, n_open_final=nof,
                               rank_bounds=(8, r + 4))


def _c128(net):
    out = dict(net)
    out["stem"] = {"labels": net["stem"]["labels"],
                   "data": np.asarray(net["stem"]["data"], dtype=np.complex128)}
    out["branches"] = [{"labels": b["labels"], "data": np.asarray(b["data"], np.complex128)}
                       for b in net["branches"]]
    return out


def _eligible(s):
    return s["cmode"] == 1 and s["K"] % 8 == 0 and s["N"] % 16 == 0 and s["M"] % 64 == 0


@pytest.mark.parametrize("cfg", NETS, ids=lambda c: f"seed{c[0]}")
def test_3m_product_matches_oracle(cfg):
    net = _net(cfg)
    onet = _c128(net)
    plan = Plan(net)
    steps = plan.steps()
    elig = [i for i, s in enumerate(steps) if _eligible(s)]
    assert elig, "no step with whole 3M tiles"
    n_sl, n_pr = len(net["sliced_labels"]), len(net["proj_labels"])
    projs = list(range(1 << n_pr))
    base = plan.contract(proj=projs).cpu().numpy()
    for tm, ntw, blocks, lds in SCHEDULES:
        print(f"network seed {cfg[0]}: 3M on steps {elig}, tm {tm} ntw {ntw} blocks {blocks} "
              f"lds {lds}", flush=True)
        for i in elig:
            info = plan.set_schedule(i, tm, ntw, blocks, lds, algo=1)
            assert info["sched_algo"] == 1
            assert info["sched_tm"] * info["sched_ntw"] <= 4
        for s in range(1 << n_sl):
            got = plan.contract(s, s + 1, proj=projs).cpu().numpy()
            for p in projs:
                ref, _ = stemnet.run_slice(onet, s, p)
                err = stats.rel_l2(got[p], ref.reshape(-1))
                assert err <= 1e-5, (s, p, err)
        tot = plan.contract(proj=projs).cpu().numpy()
        for p in projs:
            assert stats.rel_l2(tot[p], base[p]) <= 1e-5
    plan.close()


@pytest.mark.parametrize("seed", [60, 66])
def test_3m_on_batched_steps_matches_oracle(seed):
    """Hyperedge networks whose batched steps (kept shared labels) have whole
    3M tiles: each batch index runs its own 3M product."""
    net = random_stem_network(seed, stem_rank=14, n_steps=6, s_range=(3, 6), f_range=(4, 6),
                              n_sliced=1, n_proj=1, n_open_final=6, batch_prob=0.5,
                              rank_bounds=(8, 18))
    onet = _c128(net)
    plan = Plan(net)
    steps = plan.steps()
    elig = [i for i, s in enumerate(steps) if _eligible(s)]
    assert any(steps[i]["n_batch"] > 0 for i in elig)
    for tm, ntw, blocks, lds in SCHEDULES[:2]:
        print(f"network seed {seed}: 3M on steps {elig}, tm {tm} ntw {ntw} lds {lds}", flush=True)
        for i in elig:
            plan.set_schedule(i, tm, ntw, blocks, lds, algo=1)
        got = plan.contract(0, 2, proj=[0, 1]).cpu().numpy()
        for p in (0, 1):
            ref = stemnet.sliced_sum(onet, proj=p).reshape(-1)
            assert stats.rel_l2(got[p], ref) <= 1e-5, p
    plan.close()


def test_3m_refused_where_it_does_not_apply():
    net = _net(NETS[0])
    plan = Plan(net)
    steps = plan.steps()
    bad = [i for i, s in enumerate(steps) if not _eligible(s)]
    good = [i for i, s in enumerate(steps) if _eligible(s)]
    for i in bad:
        with pytest.raises(C.StemError) as e:
            plan.set_schedule(i, algo=1)
        assert e.value.status == C.STEM_EUNSUPPORTED
    with pytest.raises(C.StemError) as e:
        plan.set_schedule(good[0], tm=3)
    assert e.value.status == C.STEM_ERANGE
    with pytest.raises(C.StemError) as e:
        plan.set_schedule(len(steps))
    assert e.value.status == C.STEM_ERANGE
    plan.close()
    split = Plan(net, precision="split_fp16")
    with pytest.raises(C.StemError) as e:
        split.set_schedule(good[0], algo=1)
    assert e.value.status == C.STEM_EUNSUPPORTED
    split.close()
