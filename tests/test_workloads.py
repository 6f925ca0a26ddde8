"""Properties of the seeded input generators (no method arithmetic here)."""
import numpy as np

from workloads import circuits, tensors


def _all_couplers(rows, cols, dead=()):
    _, index = circuits.grid_sites(rows, cols, dead)
    out = set()
    for (r, c), q in index.items():
        for other in [(r, c + 1), (r + 1, c)]:
            if other in index:
                out.add(frozenset((q, index[other])))
    return out


def test_patterns_are_matchings_covering_every_coupler():
    for rows, cols, dead in [(4, 5, ()), (5, 6, ()), (6, 9, ((0, 4),))]:
        seen = []
        for letter in "ABCD":
            pairs = circuits.coupler_pattern(rows, cols, letter, dead)
            qs = [q for p in pairs for q in p]
            assert len(qs) == len(set(qs)), "pattern is not a matching"
            seen.extend(frozenset(p) for p in pairs)
        assert len(seen) == len(set(seen))
        assert set(seen) == _all_couplers(rows, cols, dead)


def test_circuit_layers_and_no_repeat_rule():
    c = circuits.make_circuit(4, 5, 8, seed=1)
    assert c["n_qubits"] == 20
    kinds = [m["kind"] for m in c["moments"]]
    assert kinds == ["1q", "2q"] * 8 + ["1q"]
    pats = "".join(m["pattern"] for m in c["moments"] if m["kind"] == "2q")
    assert pats == "ABCDCDAB"
    layers = [m["gates"] for m in c["moments"] if m["kind"] == "1q"]
    for prev, cur in zip(layers, layers[1:]):
        assert all(a != b for a, b in zip(prev, cur))
    used = {g for layer in layers for g in layer}
    assert used <= set(circuits.GATE_1Q_NAMES)


def test_circuit_is_deterministic_and_seed_dependent():
    a = circuits.make_circuit(3, 3, 5, seed=7)
    b = circuits.make_circuit(3, 3, 5, seed=7)
    c = circuits.make_circuit(3, 3, 5, seed=8)
    assert a == b and a != c


def test_53_qubit_layout():
    c = circuits.make_circuit(6, 9, 2, seed=5, dead=[(0, 4)])
    assert c["n_qubits"] == 53


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 seeded with 0 (Steele, Lea, Flood 2014;
    # the same stream as Vigna's reference splitmix64.c)
    out = tensors.splitmix64(0, np.arange(3))
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                     0x06C45D188009454F]


def test_counter_stem_entries_are_float32_exact():
    v = tensors.counter_stem_entries(3, np.arange(4096), 20)
    assert np.array_equal(v.real.astype(np.float32).astype(np.float64), v.real)
    assert np.array_equal(v.imag.astype(np.float32).astype(np.float64), v.imag)
    assert abs(v.real.mean()) < 0.05 * v.real.std()


def test_counter_stem_norm_close_to_one():
    r = 16
    e = tensors.counter_stem_default_scale(r)
    v = tensors.counter_stem_entries(11, np.arange(1 << r), e)
    assert 0.6 < np.linalg.norm(v) < 1.6


def test_isolated_stem_shapes_stay_in_window():
    spec = tensors.random_isolated_stem(24, 40, seed=3)
    rank = 24
    labels = list(spec["stem_labels"])
    for st in spec["branches"]:
        lab = st["labels"]
        shared = [x for x in lab if x in labels]
        s = len(shared)
        r = len(lab)
        assert 4 <= s <= 8 and 6 <= r <= 14
        rank = rank - s + (r - s)
        assert 22 <= rank <= 24
        labels = [x for x in labels if x not in shared] + [x for x in lab if x not in shared]
        # columns of the branch matrix have unit norm over the shared labels
        m = st["data"].reshape(1 << s, -1)
        assert np.allclose(np.linalg.norm(m, axis=0), 1.0, atol=1e-5)
    assert sorted(labels) == sorted(spec["final_labels"])


def test_bitstrings_and_prefix():
    bs = tensors.random_bitstrings(20, 64, 1001)
    assert len(bs) == 64 and all(0 <= b < (1 << 20) for b in bs)
    sp = tensors.split_open_prefix(20, [4, 3, 9, 2, 8, 7], 1001)
    assert sp["open"] == [2, 3, 4, 7, 8, 9]
    assert len(sp["closed"]) == 14 and len(sp["closed_bits"]) == 14
