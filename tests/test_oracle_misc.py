"""Pins of the dense step definitions, costs, statistics and the MLP."""
import math

import numpy as np
import pytest

from oracle import cost, dense, mlp, stats


def test_permute_labels_matches_bit_loop():
    rng = np.random.Generator(np.random.PCG64(0))
    for r in [1, 3, 6]:
        data = rng.standard_normal(1 << r) + 1j * rng.standard_normal(1 << r)
        lin = list(range(r))
        lout = [int(x) for x in rng.permutation(r)]
        assert np.array_equal(dense.permute_labels(data, lin, lout),
                              dense.permute_bits_loop(data, lin, lout))


def test_permute_known_case():
    # 2 labels: swapping them is a 2x2 transpose
    d = np.array([0, 1, 2, 3])
    assert list(dense.permute_labels(d, [0, 1], [1, 0])) == [0, 2, 1, 3]


def test_cgemm_triple_sum_and_real_embedding():
    rng = np.random.Generator(np.random.PCG64(1))
    a = rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))
    b = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    c = dense.cgemm(a, b)
    for i in range(5):
        for j in range(4):
            assert abs(c[i, j] - sum(a[i, k] * b[k, j] for k in range(3))) < 1e-12
    # real embedding: [re a, im a] (interleaved) times the 2x2 block form
    ar = np.stack([a.real, a.imag], axis=-1).reshape(5, 6)
    br = np.zeros((6, 8))
    for k in range(3):
        for n in range(4):
            br[2 * k, 2 * n], br[2 * k, 2 * n + 1] = b[k, n].real, b[k, n].imag
            br[2 * k + 1, 2 * n], br[2 * k + 1, 2 * n + 1] = -b[k, n].imag, b[k, n].real
    cr = (ar @ br).reshape(5, 4, 2)
    assert np.allclose(cr[..., 0] + 1j * cr[..., 1], c, atol=1e-12)


def test_matrix_chain_cost():
    # A(a,b) B(b,c) C(c,d), open a,d: (AB) costs 2^3, then (AB)C 2^3
    leaves = [{0, 1}, {1, 2}, {2, 3}]
    tc, cw, per = cost.scheme_cost(leaves, [(0, 1), (0, 1)], open_labels=[0, 3])
    assert per == [(3, 2), (3, 2)] and tc == 16 and cw == 2


def test_step_time_is_mkn():
    # stem with 5 free + 3 shared labels, branch with 3 shared + 2 free
    leaves = [set(range(8)), {5, 6, 7, 20, 21}]
    tc, cw, per = cost.scheme_cost(leaves, [(0, 1)], open_labels=[0, 1, 2, 3, 4, 20, 21])
    assert tc == (2 ** 5) * (2 ** 3) * (2 ** 2) and cw == 7


def test_slicing_multiplies_time():
    leaves = [{0, 1, 2}, {1, 2, 3}, {3, 0}]
    tc0, cw0, _ = cost.scheme_cost(leaves, [(0, 1), (0, 1)])
    tc1, cw1, _ = cost.scheme_cost(leaves, [(0, 1), (0, 1)], sliced=[1])
    # slicing label 1: steps cost 2^3 and 2^2 (was 2^4 and 2^2), times 2
    assert tc0 == 16 + 4 and cw0 == 2
    assert tc1 == 2 * (8 + 4) and cw1 == 2


def test_stem_scheme_steps_absorb_in_order():
    leaves = [{0, 1, 2}, {2, 3}, {3, 4}, {4, 1, 0}]
    steps = cost.stem_scheme_steps(3)
    tc, cw, per = cost.scheme_cost(leaves, steps)
    assert per == [(4, 3), (4, 3), (3, 0)]


# Table 1 of the paper: contraction cost per sample (complex MACs), one-V100
# time per perfect sample, printed FLOPS efficiency (of 15.7 TFLOP/s)
TABLE1 = [(1.09e13, 38.02, 14.56), (7.16e13, 243.71, 14.97),
          (1.15e17, 4.82 * 86400, 14.05), (2.59e17, 9.18 * 86400, 16.67),
          (6.66e18, 266.80 * 86400, 14.74)]


@pytest.mark.parametrize("macs,sec,eff", TABLE1)
def test_table1_flop_convention(macs, sec, eff):
    got = 100.0 * cost.flops(macs) / (sec * 15.7e12)
    assert abs(got - eff) < 0.1


def test_closing_estimate_of_experiments_section():
    # 8 * 10^18.6 FLOPs per sample at 90% of 15.7 TFLOP/s on 27648 GPUs,
    # 2000 samples: about 1.63e5 s (1.89 days)
    t = cost.flops(10 ** 18.6) / (15.7e12 * 0.9 * 27648) * 2000
    assert abs(t - 1.63e5) / 1.63e5 < 0.01 and abs(t / 86400 - 1.89) < 0.01


def test_xeb_special_cases():
    n = 4
    uni = np.full(16, 0.25 + 0j)  # |a|^2 = 1/16
    assert abs(stats.xeb(uni, n)) < 1e-15
    assert abs(stats.collision_xeb(uni, n)) < 1e-15
    # two states with probability 1/2 each: 2^n * mean p - 1 = 16/2 - 1 = 7
    amp = np.zeros(16, complex); amp[3] = amp[7] = math.sqrt(0.5)
    assert abs(stats.xeb(amp[[3, 7]], n) - 7.0) < 1e-12
    assert abs(stats.collision_xeb(amp, n) - 7.0) < 1e-12


def test_porter_thomas_ks_exact_quantiles():
    m = 20000
    q = -np.log(1.0 - (np.arange(m) + 0.5) / m)  # exponential quantiles
    assert stats.porter_thomas_ks(q / m, m) < 1e-3
    assert stats.porter_thomas_ks(np.full(m, 1.0 / m), m) > 0.3


def test_rel_l2():
    assert stats.rel_l2([1, 0], [1, 0]) == 0.0
    assert abs(stats.rel_l2([1, 1e-3], [1, 0]) - 1e-3) < 1e-15


def _fd_grad(params, x, t, key, eps=1e-6):
    g = np.zeros_like(params[key])
    it = np.nditer(params[key], flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        p_plus = {k: v.copy() for k, v in params.items()}
        p_minus = {k: v.copy() for k, v in params.items()}
        p_plus[key][i] += eps
        p_minus[key][i] -= eps
        g[i] = (mlp.loss(p_plus, x, t) - mlp.loss(p_minus, x, t)) / (2 * eps)
    return g


def test_mlp_gradients_match_finite_differences():
    rng = np.random.Generator(np.random.PCG64(5))
    params = mlp.init_params(6, 8, seed=3)
    for k in ("b1", "b2"):
        params[k] = rng.standard_normal(params[k].shape) * 0.1
    x = rng.standard_normal((10, 6))
    t = rng.standard_normal(10)
    _, g = mlp.backward(params, x, t)
    for key in mlp.PARAM_NAMES:
        fd = _fd_grad(params, x, t, key)
        assert np.allclose(g[key], fd, rtol=1e-5, atol=1e-7), key


def test_mlp_hand_set_weights():
    p = {"W1": np.array([[1.0, -1.0]]), "b1": np.array([0.0, 0.5]),
         "W2": np.eye(2), "b2": np.array([0.0, 0.0]),
         "W3": np.array([[2.0], [3.0]]), "b3": np.array([1.0])}
    y, _ = mlp.forward(p, np.array([[2.0], [-1.0]]))
    # x=2: h1=(2,0), h2=(2,0), y=4+1=5; x=-1: h1=(0,1.5), y=4.5+1=5.5
    assert np.allclose(y, [5.0, 5.5])


def test_adam_first_step():
    params = {k: np.ones(3) for k in mlp.PARAM_NAMES}
    grads = {k: np.array([0.5, -2.0, 0.0]) for k in mlp.PARAM_NAMES}
    state = {}
    mlp.adam_step(params, grads, state, lr=0.01, eps=1e-8)
    step = 0.01 * np.array([0.5, -2.0, 0.0]) / (np.abs([0.5, -2.0, 0.0]) + 1e-8)
    for k in mlp.PARAM_NAMES:
        assert np.allclose(params[k], 1.0 - step, atol=1e-12)


def test_frugal_sampling_special_cases():
    n = 6
    rng = np.random.Generator(np.random.PCG64(9))
    a = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    p = np.abs(a) ** 2
    p /= p.sum()
    amps = np.sqrt(p)
    # M above every N p: every candidate is accepted with probability N p / M,
    # the accepted ones follow p, and their XEB is the collision XEB
    big = 2.0 * p.max() * p.size
    assert stats.frugal_xeb(p, big) == pytest.approx(stats.collision_xeb(amps, n), rel=1e-12)
    assert stats.frugal_acceptance(p, big) == pytest.approx(1.0 / big, rel=1e-12)
    # M below every N p: every candidate is accepted, uniform samples, XEB 0
    small = 0.5 * p.min() * p.size
    assert abs(stats.frugal_xeb(p, small)) < 1e-12
    assert stats.frugal_acceptance(p, small) == 1.0
    # two outcomes, p = (0.9, 0.1), N = 2, M = 1: q = (0.5, 0.1) / 0.6,
    # XEB = 2 (0.5 * 0.9 + 0.1 * 0.1) / 0.6 - 1 = 8/15; acceptance (1 + 0.2) / 2
    two = np.array([0.9, 0.1])
    assert stats.frugal_xeb(two, 1.0) == pytest.approx(8.0 / 15.0, rel=1e-12)
    assert stats.frugal_acceptance(two, 1.0) == pytest.approx(0.6, rel=1e-12)
