"""Pins for the measure of importance (Eq. 1) and the weighted sampler (Sec. 3.1)."""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import sambaten as sb


def test_moi_scale_headroom():
    for max_x2, n_max in [(1.0, 1000), (3.7, 123457), (1e-6, 10 ** 9), (250.0, 7)]:
        S = sb.moi_scale(max_x2, n_max)
        assert math.ldexp(max_x2, S) * n_max < 2.0 ** 58
        assert math.ldexp(max_x2, S) * n_max >= 2.0 ** 56
    assert sb.moi_scale(0.0, 10) == 32


def test_quantized_moi_equals_exact_fraction_sums():
    g = np.random.default_rng(0)
    X = (g.standard_normal((4, 3, 5)) * 3).astype(np.float32)
    S = sb.moi_scale(float(np.max(X.astype(np.float64) ** 2)), 60)
    q, ok = sb.quantize_sq(X, S, 60)
    assert ok
    w1, w2, w3 = sb.moi_dense(q)
    I, J, K = X.shape
    for i in range(I):
        exact = sum(math.floor(Fraction(float(X[i, j, k])) ** 2 * Fraction(2) ** S)
                    for j in range(J) for k in range(K))
        assert int(w1[i]) == exact
    for j in range(J):
        exact = sum(math.floor(Fraction(float(X[i, j, k])) ** 2 * Fraction(2) ** S)
                    for i in range(I) for k in range(K))
        assert int(w2[j]) == exact
    for k in range(K):
        exact = sum(math.floor(Fraction(float(X[i, j, k])) ** 2 * Fraction(2) ** S)
                    for i in range(I) for j in range(J))
        assert int(w3[k]) == exact


def test_moi_proportional_to_sum_of_squares():
    # Eq. 1: x_a(i) = sum_jk X(i,j,k)^2; the integer form is that times 2^S, floored per entry
    g = np.random.default_rng(1)
    X = g.standard_normal((6, 5, 4)).astype(np.float32)
    S = sb.moi_scale(float(np.max(X.astype(np.float64) ** 2)), 120)
    q, _ = sb.quantize_sq(X, S, 120)
    w1, w2, w3 = sb.moi_dense(q)
    X64 = X.astype(np.float64)
    for w, ref in ((w1, (X64 ** 2).sum(axis=(1, 2))), (w2, (X64 ** 2).sum(axis=(0, 2))),
                   (w3, (X64 ** 2).sum(axis=(0, 1)))):
        np.testing.assert_allclose(w.astype(np.float64) * 2.0 ** -S, ref, rtol=1e-12, atol=0)


def test_moi_coo_permutation_invariant_and_equals_dense():
    g = np.random.default_rng(2)
    X = g.standard_normal((6, 5, 4)).astype(np.float32)
    X[np.abs(X) < 0.8] = 0
    idx = np.argwhere(X != 0)
    vals = X[X != 0]
    S = 20
    q, _ = sb.quantize_sq(vals, S, 120)
    qd, _ = sb.quantize_sq(X, S, 120)
    dense = sb.moi_dense(qd)
    coo = sb.moi_coo(idx, q, X.shape)
    perm = g.permutation(len(vals))
    coo_p = sb.moi_coo(idx[perm], q[perm], X.shape)
    for a, b, c in zip(dense, coo, coo_p):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(b, c)


def test_quantize_rejects_overflow_and_nonfinite():
    _, ok = sb.quantize_sq(np.array([1.0, np.nan]), 10, 100)
    assert not ok
    _, ok = sb.quantize_sq(np.array([np.inf]), 10, 100)
    assert not ok
    S = sb.moi_scale(1.0, 100)
    _, ok = sb.quantize_sq(np.array([1.0]), S, 100)
    assert ok
    _, ok = sb.quantize_sq(np.array([200.0]), S, 100)  # x^2 * 2^S > 2^63 / N_max
    assert not ok


def test_sample_all_when_n_equals_N():
    w = np.array([5, 0, 3, 9, 1], dtype=np.uint64)
    np.testing.assert_array_equal(sb.sample_mode(w, 5, 1, 0, 1, 0, 0), np.arange(5))


def test_sample_sorted_unique_and_deterministic():
    w = np.random.default_rng(3).integers(1, 1000, size=300).astype(np.uint64)
    a = sb.sample_mode(w, 40, 7, 2, 2, 3, 4)
    b = sb.sample_mode(w, 40, 7, 2, 2, 3, 4)
    np.testing.assert_array_equal(a, b)
    assert len(a) == 40 and np.all(np.diff(a) > 0)
    c = sb.sample_mode(w, 40, 7, 2, 2, 3, 5)   # next batch counter
    d = sb.sample_mode(w, 40, 7, 2, 2, 4, 4)   # next repetition
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_zero_weight_never_chosen_while_positive_remain():
    w = np.zeros(50, dtype=np.uint64)
    w[[3, 17, 20, 41]] = [1, 2, 3, 4]
    for t in range(50):
        s = sb.sample_mode(w, 4, 1, 0, 1, 0, t)
        np.testing.assert_array_equal(s, [3, 17, 20, 41])
    # more draws than positive weights: zeros are taken last, by index
    s = sb.sample_mode(w, 6, 1, 0, 1, 0, 0)
    np.testing.assert_array_equal(s, [0, 1, 3, 17, 20, 41])
    np.testing.assert_array_equal(sb.sample_mode(np.zeros(9, np.uint64), 3, 1, 0, 1, 0, 0),
                                  [0, 1, 2])


def test_dominant_weight_always_chosen():
    w = np.ones(40, dtype=np.uint64)
    w[29] = 1 << 40
    for t in range(100):
        assert 29 in sb.sample_mode(w, 2, 2, 0, 3, 1, t)


def test_uniform_weights_inclusion_probability():
    N, n, T = 40, 10, 1500
    w = np.full(N, 7, dtype=np.uint64)
    counts = np.zeros(N)
    for t in range(T):
        counts[sb.sample_mode(w, n, 11, 0, 1, 0, t)] += 1
    expected = T * n / N
    chi2 = float(np.sum((counts - expected) ** 2 / expected))
    # chi-square with 39 dof (slightly conservative: without-replacement draws)
    assert chi2 < 80.0


def successive_sampling_probs(w, n):
    """Exact probability of each n-subset under draw-proportional-to-remaining-weight."""
    N = len(w)
    W = float(sum(w))
    probs = {}
    for perm in itertools.permutations(range(N), n):
        p, rem = 1.0, W
        for i in perm:
            p *= w[i] / rem
            rem -= w[i]
        key = tuple(sorted(perm))
        probs[key] = probs.get(key, 0.0) + p
    return probs


@pytest.mark.parametrize("w,n", [([1, 2, 3, 4, 10], 2), ([5, 1, 1, 8], 3), ([2, 9, 4], 1)])
def test_exponential_keys_are_successive_sampling(w, n):
    exact = successive_sampling_probs(w, n)
    T = 6000
    wa = np.array(w, dtype=np.uint64)
    counts = {}
    for t in range(T):
        key = tuple(int(v) for v in sb.sample_mode(wa, n, 5, 0, 2, 1, t))
        counts[key] = counts.get(key, 0) + 1
    for key, p in exact.items():
        freq = counts.get(key, 0) / T
        sd = math.sqrt(p * (1 - p) / T)
        assert abs(freq - p) < 5 * sd + 1e-3, (key, freq, p)
    # a with-replacement or inclusion-proportional scheme would put mass elsewhere:
    # every observed subset must be one the exact enumeration allows
    assert set(counts) <= set(exact)


def test_sample_size_is_the_ceiling_for_ragged_ratios():
    # n = ceil(N / s) (Sec. 3.1 samples a 1/s fraction of each mode; the rounding
    # is the reading taken): the smallest n with n * s >= N, at least 1 and at
    # most N.  Checked by counting up rather than by a formula, over ragged and
    # exact ratios, s larger than N and s = 1.
    for N in list(range(1, 40)) + [99, 100, 101, 997, 100000, 100001]:
        for s in (1, 2, 3, 5, 7, 10, 16, 41, 1000):
            n = 1
            while n * s < N:
                n += 1
            assert sb.sample_size(N, s) == min(n, N), (N, s)
    # a floor slip would give 0 or N // s here
    assert sb.sample_size(11, 5) == 3 and sb.sample_size(4, 5) == 1
    assert sb.sample_size(100001, 10) == 10001
