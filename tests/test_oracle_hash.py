"""Pins of the oracle's hash-generated CountSketch (the future-work variant of
Sec. 8: bucket and sign of row i computed from (seed, i), no stored h and s).

The generator is SplitMix64, pinned to its published known answers
(tests/golden/splitmix64_kat.txt).  The map from an output u to (h, s) is
pinned by special cases with a plain definition (k a power of two: h is the
top log2(k) bits of u; k = 1: every h is 0), by range, uniformity and sign
balance, and by the CountSketch of the generated (h, s) against the dense
sketch matrix of Def. 3.
"""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_kat.txt")


def _kat():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        seed, vals = line.split(";")
        out.append((int(seed.strip(), 0), [int(v.strip(), 0) for v in vals.split(",")]))
    return out


@pytest.mark.parametrize("seed,expect", _kat())
def test_splitmix64_known_answers(orc, seed, expect):
    got = orc.splitmix64(seed, len(expect))
    assert [int(x) for x in got] == expect


def test_hash_sketch_row_i_is_output_i_plus_1(orc):
    # row i takes the (i+1)-th output; with k = 2^m, h is the top m bits of it
    # and s the sign of its bit 0
    seed, d = 987654321, 3000
    u = orc.splitmix64(seed, d)
    for m in (0, 1, 7, 13, 31):
        h, s = orc.hash_sketch(d, 1 << m, seed)
        top = (u >> np.uint64(64 - m)).astype(np.int64) if m else np.zeros(d, dtype=np.int64)
        assert np.array_equal(h.astype(np.int64), top)
        assert np.array_equal(s, np.where((u & np.uint64(1)) == 1, -1, 1).astype(np.int8))


def test_hash_sketch_range_uniformity_balance(orc):
    d, k = 200000, 1000
    h, s = orc.hash_sketch(d, k, 14209)
    assert h.min() >= 0 and h.max() < k
    assert set(np.unique(s)) == {-1, 1}
    cnt = np.bincount(h, minlength=k)
    chi2 = float(((cnt - d / k) ** 2 / (d / k)).sum())
    # chi-square with 999 degrees of freedom: mean 999, sd ~ 44.7
    assert 999 - 6 * 44.7 < chi2 < 999 + 6 * 44.7
    # signs: +1 with probability 1/2 (6 standard deviations)
    assert abs(int(s.sum())) < 6 * np.sqrt(d)
    # sign independent of the bucket parity
    odd = h % 2 == 1
    assert abs(int(s[odd].sum())) < 6 * np.sqrt(odd.sum())


def test_hash_sketch_seeds_and_prefixes(orc):
    h1, s1 = orc.hash_sketch(5000, 777, 1)
    h2, s2 = orc.hash_sketch(5000, 777, 2)
    assert np.mean(h1 == h2) < 0.01
    # a row's (h, s) depends on (seed, i) only, not on d
    h3, s3 = orc.hash_sketch(123, 777, 1)
    assert np.array_equal(h3, h1[:123]) and np.array_equal(s3, s1[:123])


def test_countsketch_hashed_is_def3_with_generated_vectors(orc):
    rng = np.random.default_rng(3)
    d, n, k, seed = 700, 5, 37, 424242
    A = np.asfortranarray(rng.integers(-8, 9, size=(d, n)).astype(np.float64))
    h, s = orc.hash_sketch(d, k, seed)
    S = np.zeros((k, d))
    S[h, np.arange(d)] = s
    assert np.array_equal(orc.countsketch_hashed(A, k, seed), S @ A)
