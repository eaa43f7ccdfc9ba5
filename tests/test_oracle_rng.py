"""Pins for the oracle's random numbers and logarithm (Sec. 3.1 sampling)."""

import math
import os

import numpy as np

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def load_kat():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(w, 16) for w in line.split()])
    return rows


def test_philox_known_answers():
    rows = load_kat()
    assert len(rows) == 3
    for r in rows:
        out = rng.philox4x32_10(*r[:6])
        assert [int(o) for o in out] == r[6:]


def test_philox_vectorised_equals_scalar():
    c0 = np.arange(100, dtype=np.uint64)
    v = rng.philox4x32_10(c0, 7, 0x01200003, 5, 123, 456)
    for i in (0, 1, 57, 99):
        s = rng.philox4x32_10(i, 7, 0x01200003, 5, 123, 456)
        assert [int(x[i]) for x in v] == [int(x) for x in s]


def test_uniform_open_exact_grid():
    u = rng.bits64(9, 1, np.arange(10000, dtype=np.uint64), 0, 77, 3)
    U = rng.uniform_open(u)
    assert np.all(U > 0) and np.all(U < 1)
    k = U * 2.0 ** 53
    assert np.all(k == np.round(k)) and np.all(k.astype(np.int64) % 2 == 1)
    assert rng.uniform_open(np.uint64(0)) == 2.0 ** -53
    assert rng.uniform_open(np.uint64(0xFFFFFFFFFFFFFFFF)) == 1.0 - 2.0 ** -53


def test_uniform_closed0_range_and_mean():
    u = rng.bits64(1, 0, np.arange(200000, dtype=np.uint64), 3, 5, 0)
    U = rng.uniform_closed0(u)
    assert U.min() >= 0 and U.max() < 1
    assert abs(U.mean() - 0.5) < 4 * math.sqrt(1 / 12 / U.size)


def test_ln_basic_accuracy_and_special_values():
    u = rng.bits64(3, 0, np.arange(1_000_000, dtype=np.uint64), 0, 1, 0)
    U = rng.uniform_open(u)
    L = rng.ln_basic(U)
    ref = np.log(U)
    ulp = np.spacing(np.abs(ref))
    assert np.max(np.abs(L - ref) / ulp) <= 4.0
    assert rng.ln_basic(np.array([1.0]))[0] == 0.0
    assert rng.ln_basic(np.array([0.5]))[0] == -rng.LN2
    assert rng.ln_basic(np.array([2.0 ** -53]))[0] == -53 * rng.LN2
    # the sqrt(2) split point on both sides
    for x in (rng.SQRT2, np.nextafter(rng.SQRT2, 2.0), 0.5 * rng.SQRT2):
        assert abs(rng.ln_basic(np.array([x]))[0] - math.log(x)) <= 4 * math.ulp(abs(math.log(x)))


def test_ln_basic_monotone():
    U = np.sort(rng.uniform_open(rng.bits64(4, 0, np.arange(200000, dtype=np.uint64), 0, 2, 0)))
    L = rng.ln_basic(U)
    assert np.all(np.diff(L) >= 0)


def test_exponential_variate_moments():
    E = rng.exp_variate(rng.bits64(5, 0, np.arange(400000, dtype=np.uint64), 0, 4, 1))
    assert np.all(E > 0)
    assert abs(E.mean() - 1.0) < 5 / math.sqrt(E.size)
    assert abs(E.var() - 1.0) < 0.02
