"""Pins for the oracle's CountSketch, bucket histogram and sketch plan.

Each check is fixed by something other than the oracle: the dense matrix S of
Def. 3 multiplied by a library matmul, hand-worked IEEE folds, invariants of
Def. 3, a closed-form second moment, and library histogram/sort routines.
"""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "canonical_fold.txt")


def dense_sketch(h, s, k):
    """S in R^{k x d} built column by column from Def. 3: s_j = sigma_j e_{r_j}."""
    d = h.shape[0]
    S = np.zeros((k, d))
    S[h, np.arange(d)] = s
    return S


def int_matrix(d, n, seed, lo=-1000, hi=1000):
    g = np.random.default_rng(seed)
    return np.asfortranarray(g.integers(lo, hi, size=(d, n)).astype(np.float64))


@pytest.mark.parametrize("d,n,k", [(1, 1, 1), (7, 3, 4), (300, 5, 17), (2048, 9, 64)])
def test_dense_brute_force_integer_exact(orc, d, n, k):
    # integer-valued A: every summation order gives the exact sum, so the
    # oracle must agree bit for bit with the dense product S A.
    h = synth.bucket_map(d, k, seed=d + k)
    s = synth.signs(d, seed=d + k)
    A = int_matrix(d, n, seed=d)
    Y = orc.countsketch(A, h, s, k)
    ref = dense_sketch(h, s, k) @ A
    assert np.array_equal(Y, ref)
    Y32 = orc.countsketch(A.astype(np.float32), h, s, k)
    assert np.array_equal(Y32, ref.astype(np.float32))


def test_dense_brute_force_gaussian(orc):
    d, n, k = 5000, 6, 128
    h = synth.bucket_map(d, k, seed=1)
    s = synth.signs(d, seed=1)
    A = synth.normal_matrix(d, n, seed=1)
    Y = orc.countsketch(A, h, s, k)
    ref = dense_sketch(h, s, k) @ A
    # the only difference is the association order of at most ~d/k terms
    assert np.linalg.norm(Y - ref) <= 1e-14 * np.linalg.norm(ref)


def test_sketch_of_identity_is_S(orc):
    d, k = 257, 31
    h = synth.bucket_map(d, k, seed=3)
    s = synth.signs(d, seed=3)
    S = orc.countsketch(np.eye(d), h, s, k)
    # exactly one +-1 per column, at row h[i] with sign s[i] (Def. 3)
    assert np.array_equal(np.count_nonzero(S, axis=0), np.ones(d))
    assert np.array_equal(np.abs(S).sum(axis=0), np.ones(d))
    assert np.array_equal(S[h, np.arange(d)], s.astype(np.float64))


def test_k_equals_one_is_signed_column_sum(orc):
    d, n = 999, 4
    A = int_matrix(d, n, seed=5)
    s = synth.signs(d, seed=5)
    Y = orc.countsketch(A, np.zeros(d, np.int32), s, 1)
    assert np.array_equal(Y[0], s.astype(np.float64) @ A)


def test_permutation_bucket_map_is_signed_row_permutation(orc):
    d, n = 300, 5
    A = synth.normal_matrix(d, n, seed=6)
    h = np.random.default_rng(6).permutation(d).astype(np.int32)
    s = synth.signs(d, seed=6)
    Y = orc.countsketch(A, h, s, d)
    expect = np.empty_like(A)
    expect[h] = s[:, None] * A
    assert np.array_equal(Y, expect)


def test_linearity_exact_for_powers_of_two(orc):
    d, n, k = 4000, 3, 50
    h = synth.bucket_map(d, k, seed=7)
    s = synth.signs(d, seed=7)
    A1 = int_matrix(d, n, seed=71)
    A2 = int_matrix(d, n, seed=72)
    lhs = orc.countsketch(4.0 * A1 - 0.5 * A2, h, s, k)
    rhs = 4.0 * orc.countsketch(A1, h, s, k) - 0.5 * orc.countsketch(A2, h, s, k)
    assert np.array_equal(lhs, rhs)


def test_row_permutation_invariance(orc):
    d, n, k = 3000, 4, 40
    h = synth.bucket_map(d, k, seed=8)
    s = synth.signs(d, seed=8)
    A = int_matrix(d, n, seed=8)
    p = np.random.default_rng(8).permutation(d)
    assert np.array_equal(orc.countsketch(A, h, s, k),
                          orc.countsketch(A[p], h[p], s[p], k))


def test_empty_buckets_are_positive_zero(orc):
    d, k = 10, 100
    h = np.arange(d, dtype=np.int32) * 3
    s = np.ones(d, np.int8)
    Y = orc.countsketch(-np.zeros((d, 2)), h, s, k)
    assert not np.signbit(Y).any()


def _golden_cases():
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        dt, vals, expect = [t.strip() for t in line.split(";")]
        yield dt, [float(v) for v in vals.split(",")], float(expect)


@pytest.mark.parametrize("case", list(_golden_cases()))
def test_canonical_fold_order_golden(orc, case):
    dt, vals, expect = case
    dtype = np.float64 if dt == "f64" else np.float32
    # put the bucket-0 rows among decoys in other buckets, signs split between
    # the stored value and s so that both paths of Alg. 2 are exercised
    d = 3 * len(vals)
    A = np.ones((d, 1), dtype=dtype)
    h = np.ones(d, np.int32)
    s = np.ones(d, np.int8)
    for j, v in enumerate(vals):
        i = 3 * j + 1
        h[i] = 0
        if j % 2:
            A[i, 0], s[i] = -v, -1
        else:
            A[i, 0], s[i] = v, 1
    Y = orc.countsketch(A, h, s, 2)
    assert Y.dtype == dtype
    got = float(Y[0, 0])
    assert got == expect and np.signbit(got) == np.signbit(expect)


def test_second_moment_closed_form(orc):
    # E||S y||^2 = ||y||^2 and Var = (2/k)(||y||^4 - ||y||_4^4) (Def. 3 with
    # independent Rademacher signs and uniform buckets); y has a non-zero mean
    # so a sign mistake would show up as a large bias.
    d, k, T = 2000, 64, 400
    y = 1.0 + synth.normal_matrix(d, 1, seed=11)[:, 0]
    ny2 = float(y @ y)
    var = 2.0 / k * (ny2 ** 2 - float(np.sum(y ** 4)))
    vals = []
    for t in range(T):
        h = synth.bucket_map(d, k, seed=1000 + t)
        s = synth.signs(d, seed=1000 + t)
        Y = orc.countsketch(y.reshape(-1, 1), h, s, k)
        vals.append(float(Y[:, 0] @ Y[:, 0]))
    vals = np.array(vals)
    assert abs(vals.mean() - ny2) <= 4.0 * np.sqrt(var / T)
    assert 0.6 < vals.var(ddof=1) / var < 1.5


def test_range_errors(orc):
    A = np.ones((4, 1))
    with pytest.raises(orc.OracleError) as e:
        orc.countsketch(A, np.array([0, 1, 4, 0], np.int32), np.ones(4, np.int8), 4)
    assert e.value.code == orc.ERR_RANGE
    with pytest.raises(orc.OracleError) as e:
        orc.countsketch(A, np.array([0, 1, 2, -1], np.int32), np.ones(4, np.int8), 4)
    assert e.value.code == orc.ERR_RANGE
    with pytest.raises(orc.OracleError) as e:
        orc.countsketch(A, np.zeros(4, np.int32), np.array([1, 0, 1, 1], np.int8), 4)
    assert e.value.code == orc.ERR_RANGE


@pytest.mark.parametrize("d,k", [(0, 5), (1, 1), (1000, 7), (65536, 2048)])
def test_histogram_matches_bincount(orc, d, k):
    h = synth.bucket_map(d, k, seed=12)
    cnt = orc.bucket_hist(h, k)
    assert cnt.sum() == d
    assert np.array_equal(cnt, np.bincount(h, minlength=k))


@pytest.mark.parametrize("d,k", [(0, 3), (1, 1), (5000, 37), (65536, 2048)])
def test_plan_matches_stable_argsort(orc, d, k):
    h = synth.bucket_map(d, k, seed=13)
    off, perm = orc.bucket_plan(h, k)
    assert np.array_equal(perm, np.argsort(h, kind="stable"))
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(np.bincount(h, minlength=k))]))
    for m in range(min(k, 50)):
        seg = perm[off[m]:off[m + 1]]
        assert np.all(h[seg] == m) and np.all(np.diff(seg) > 0)


def test_bucket_uniformity_chi2():
    # the bucket generator is uniform on {0..k-1} (Def. 3): chi-square test
    d, k = 1 << 20, 256
    cnt = np.bincount(synth.bucket_map(d, k, seed=14), minlength=k)
    e = d / k
    chi2 = float(((cnt - e) ** 2 / e).sum())
    # df = 255: mean 255, sd ~ 22.6; 6 sd either side
    assert 255 - 6 * 22.6 < chi2 < 255 + 6 * 22.6
    s = synth.signs(d, seed=14)
    assert set(np.unique(s)) == {-1, 1} and abs(int(s.astype(np.int64).sum())) < 6 * np.sqrt(d)


# --- FP32 data folded in FP64 (the "plain FP64" reading of an FP32 matrix) ---

def test_f32_acc64_equals_f64_fold_of_promoted_data(orc):
    # Promoting FP32 to FP64 is exact, so Def. 3 folded in FP64 over the FP32
    # values and over their FP64 images is the same computation: bit-equal.
    d, n, k = 6000, 5, 96
    h = synth.bucket_map(d, k, seed=21)
    s = synth.signs(d, seed=21)
    A32 = synth.normal_matrix(d, n, seed=21).astype(np.float32)
    Y = orc.countsketch(A32, h, s, k, acc="f64")
    assert Y.dtype == np.float64
    ref = orc.countsketch(A32.astype(np.float64), h, s, k)
    assert np.array_equal(Y.view(np.uint64), ref.view(np.uint64))


def test_f32_acc64_dense_brute_force_beyond_float_precision(orc):
    # Integer-valued FP32 entries near 2^23: every partial sum of a bucket is
    # an integer below 2^53, so the FP64 fold is exact and must equal the dense
    # S of Def. 3 times A; the same sums overflow FP32's 24-bit significand, so
    # a fold in float (or a dropped or flipped sign) cannot match.
    d, n, k = 4096, 3, 8
    h = synth.bucket_map(d, k, seed=22)
    s = synth.signs(d, seed=22)
    g = np.random.default_rng(22)
    A = ((1 << 23) + g.integers(0, 1 << 20, size=(d, n))).astype(np.float32)
    Y = orc.countsketch(A, h, s, k, acc="f64")
    exact = dense_sketch(h, s, k).astype(np.int64) @ A.astype(np.int64)
    assert np.array_equal(Y, exact.astype(np.float64))
    Y32 = orc.countsketch(A, h, s, k).astype(np.float64)
    assert not np.array_equal(Y32, Y)   # the float fold does round here


def test_f32_acc64_keeps_small_terms(orc):
    # 1 + 2^-30 - 1 in one bucket: FP64 keeps 2^-30 (an FP32 fold would give
    # 0); the rows of the other bucket, signs included, give -(3 + 2^-29).
    A = np.array([[1.0], [2.0 ** -30], [3.0], [-1.0], [2.0 ** -29]], np.float32)
    h = np.array([0, 0, 1, 0, 1], np.int32)
    s = np.array([1, 1, -1, 1, -1], np.int8)
    Y = orc.countsketch(A, h, s, 2, acc="f64")
    assert Y[0, 0] == 2.0 ** -30
    assert Y[1, 0] == -(3.0 + 2.0 ** -29)


@pytest.mark.parametrize("threads", [2, 3, 8, 64])
def test_column_parallel_fold_bit_identical(orc, threads):
    # the all-cores timing variant folds each column on one thread in the
    # canonical order: bit for bit the sequential fold (including with more
    # threads than columns, and for rounding-sensitive data)
    d, n, k = 20000, 7, 300
    h = synth.bucket_map(d, k, seed=41)
    s = synth.signs(d, seed=41)
    A = synth.normal_matrix(d, n, seed=41) * np.logspace(0, 12, n)[None, :]
    ref = orc.countsketch(A, h, s, k)
    Y = orc.countsketch(A, h, s, k, threads=threads)
    assert np.array_equal(Y.view(np.uint64), ref.view(np.uint64))
    hb = h.copy()
    hb[5] = k
    with pytest.raises(orc.OracleError):
        orc.countsketch(A, hb, s, k, threads=threads)
