"""Pins for the oracle's random stream and sampler (Alg. 2 sampling step)."""

import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, philox_word0
from oracle.sampler import fixed_point_weights, sample_block, top_b, REJECTION_FACTOR
from workloads import example23

MASK = (1 << 64) - 1


def _numpy_philox(counter, key):
    """NumPy's Philox4x64-10 (an independent implementation).  NumPy adds one
    to the 256-bit little-endian counter before generating a block, so it is
    started at counter - 1."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(counter)) - 1
    v %= 1 << 256
    nc = np.array([(v >> (64 * i)) & MASK for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(counter=nc, key=np.array(key, dtype=np.uint64))
    return [int(g.random_raw()) for _ in range(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 9, 0), (123, 0)),
    ((MASK, 3, 0, 0), ((1 << 63) + 5, 17)),
    ((12345, 678, 91011, 1213), (MASK, MASK)),
])
def test_philox_matches_numpy(counter, key):
    assert list(philox4x64_10(counter, key)) == _numpy_philox(counter, key)


def test_philox_word0_counter_layout():
    # candidate j, block t, id: counter (j, t, id, 0), key (seed, 0)
    assert philox_word0(3, 5, 7, 11) == _numpy_philox((3, 5, 7, 0), (11, 0))[0]


def test_weights_are_exact_power_of_two_scaling():
    rng = np.random.default_rng(0)
    d = rng.exponential(size=1000) * 10.0 ** rng.integers(-20, 5, size=1000)
    d[::17] = 0.0
    d[5] = -1e-30                                   # rounding-negative residual
    w, s = fixed_point_weights(d)
    assert w.dtype == np.uint64
    total = sum(int(x) for x in w)
    assert total < 2 ** 62
    for i in range(0, 1000, 7):
        exact = Fraction(max(d[i], 0.0)) * (Fraction(2) ** s)
        assert int(w[i]) == math.floor(exact)
    assert w[5] == 0
    # the largest weight uses the top bits: 2^(61 - ceil log2 m) <= max w
    assert int(w.max()) >= 2 ** (61 - 10)


def test_weights_excluded_rows_are_zero():
    d = np.arange(1.0, 11.0)
    ex = np.zeros(10, dtype=bool)
    ex[[9, 3]] = True
    w, _ = fixed_point_weights(d, ex)
    assert w[9] == 0 and w[3] == 0 and np.all(w[[0, 1, 2, 4, 5, 6, 7, 8]] > 0)


def test_draw_is_smallest_prefix_above_target_bruteforce():
    # each draw maps a word x to floor(x W / 2^64) and picks min{i : C_i > target}
    rng = np.random.default_rng(1)
    d = rng.uniform(size=37)
    d[[3, 4, 20]] = 0.0
    w, _ = fixed_point_weights(d)
    C = np.cumsum(w, dtype=np.uint64)
    W = int(C[-1])
    from oracle.sampler import _draw
    for j in range(200):
        x = philox_word0(j, 1, 0, 99)
        target = (x * W) >> 64
        lin = next(i for i in range(37) if int(C[i]) > target)
        assert _draw(C, x) == lin
        assert w[lin] > 0


def test_weights_below_resolution_are_zero():
    # w_i = floor(d_i 2^s) with 2^s ~ 2^(61 - ceil log2 m) / dmax: rows far
    # below the largest residual norm get no probability mass
    d = np.array([2.0 ** 60, 1.0, 1.0, 1.0, 1.0])
    w, s = fixed_point_weights(d)
    assert s == 62 - 61 - 3
    assert list(w[1:]) == [0, 0, 0, 0]
    assert sample_block(d, None, 3, seed=1, t=1) == [0]


def test_few_positive_rows_taken_in_index_order():
    d = np.zeros(50)
    d[[40, 7, 13]] = [1.0, 2.0, 3.0]
    assert sample_block(d, None, 5, seed=1, t=1) == [7, 13, 40]
    assert sample_block(d, None, 3, seed=1, t=1) == [7, 13, 40]


def test_block_is_distinct_and_positive():
    rng = np.random.default_rng(2)
    d = rng.exponential(size=500)
    d[rng.integers(0, 500, size=100)] = 0.0
    ex = np.zeros(500, dtype=bool)
    ex[rng.integers(0, 500, size=30)] = True
    for t in range(1, 6):
        S = sample_block(d, ex, 64, seed=5, t=t)
        assert len(S) == 64 and len(set(S)) == 64
        assert all(d[i] > 0 and not ex[i] for i in S)


def test_first_draw_frequencies_follow_squared_norms():
    # eq. squared_norm_distribution: P(i) = d_i / ||d||_1 (chi-square test)
    d = np.array([1.0, 2.0, 3.0, 4.0, 0.5, 7.0, 0.0, 2.5])
    counts = np.zeros(len(d))
    n_draw = 20000
    for t in range(1, n_draw + 1):
        counts[sample_block(d, None, 1, seed=3, t=t)[0]] += 1
    p = d / d.sum()
    keep = p > 0
    chi2, pval = stats.chisquare(counts[keep], n_draw * p[keep])
    assert counts[6] == 0
    assert pval > 1e-4, (counts, chi2)


def test_second_draw_is_successive_sampling():
    # without replacement: P(first=i, second=j) = p_i p_j / (1 - p_i)
    d = np.array([1.0, 2.0, 3.0, 4.0])
    p = d / d.sum()
    n_draw = 20000
    counts = {}
    for t in range(1, n_draw + 1):
        i, j = sample_block(d, None, 2, seed=4, t=t)
        counts[(i, j)] = counts.get((i, j), 0) + 1
    pairs = [(i, j) for i in range(4) for j in range(4) if i != j]
    obs = np.array([counts.get(q, 0) for q in pairs], dtype=float)
    exp = np.array([p[i] * p[j] / (1 - p[i]) for i, j in pairs]) * n_draw
    _, pval = stats.chisquare(obs, exp)
    assert pval > 1e-4


def test_removal_form_after_rejection_budget():
    # one row carries almost all the weight: the rejection budget J_max = 32 b
    # is spent, the rest are drawn with the accepted rows removed.
    d = np.array([2.0 ** 40, 1.0, 1.0, 1.0, 1.0])
    w, _ = fixed_point_weights(d)
    assert np.all(w[1:] == w[1]) and w[1] > 0
    firsts = np.zeros(5)
    for t in range(1, 801):
        S = sample_block(d, None, 3, seed=8, t=t)
        assert S[0] == 0 and len(set(S)) == 3
        firsts[S[1]] += 1
    # the second index is uniform over rows 1..4 once row 0 is removed
    _, pval = stats.chisquare(firsts[1:], np.full(4, 200.0))
    assert pval > 1e-4
    assert REJECTION_FACTOR == 32


def test_example23_closed_form_probabilities():
    # Example 2.3: p = alpha / ((alpha + beta) r) for each of the r heavy
    # directions and 1 / ((alpha + beta) r) for each light one (k = (1+beta) r)
    r, beta, alpha = 3, 2, 1.0e4
    k = (1 + beta) * r
    m = 4 * k
    X = example23(m, k, r, alpha)
    d = (X * X).sum(1)
    w, _ = fixed_point_weights(d)
    W = float(w.sum())
    rep = m // k
    for i in range(k):
        mass = float(w[i * rep:(i + 1) * rep].sum()) / W
        want = alpha / ((alpha + beta) * r) if i < r else 1.0 / ((alpha + beta) * r)
        assert abs(mass - want) <= 1e-12
    # eta_r = beta / (alpha + beta) (relative rank-r tail, eq. relative_tail)
    s = np.linalg.svd(X, compute_uv=False)
    eta = (s[r:] ** 2).sum() / (s ** 2).sum()
    assert abs(eta - beta / (alpha + beta)) <= 1e-12


def test_top_b_greedy_order():
    d = np.array([3.0, 5.0, 5.0, 0.0, 1.0, 4.0])
    ex = np.array([False, False, False, False, False, True])
    assert top_b(d, ex, 3) == [1, 2, 0]
    assert top_b(d, ex, 10) == [1, 2, 0, 4]
