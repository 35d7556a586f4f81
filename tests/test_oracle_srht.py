"""Pins of the oracle's SRHT (Sec. 5's definition, S = k^{-1/2} P H_m D) and
of the Count + SRHT multisketch (Sec. 8's future-work variant).

The Hadamard matrix is pinned to the recursive definition through SciPy's
Sylvester construction (the same recursion), and the transform to the
paper's radix-4 FWHT (Alg. 3), run here in plain Python; orthogonality,
zero padding, sampling, the norm in expectation, and the sketch-and-solve
special case with an orthogonal sketch (LAPACK least squares) complete the
pins.
"""
import numpy as np
import pytest
import scipy.linalg


def fwht_rad4(a):
    """Alg. 3 (radix-4 FWHT, in place, 0-based indices), for len(a) = 4^p."""
    a = np.array(a, dtype=np.float64)
    d = a.shape[0]
    stride = d // 4
    while stride >= 1:
        s = stride * 4
        for b in range(0, d, s):
            for kk in range(stride):
                i0 = b + kk
                i1, i2, i3 = i0 + stride, i0 + 2 * stride, i0 + 3 * stride
                x, y, z, t = a[i0], a[i1], a[i2], a[i3]
                X, Y, Z, T = x + z, y + t, x - z, y - t
                a[i0], a[i1], a[i2], a[i3] = X + Y, X - Y, Z + T, Z - T
        stride //= 4
    return a


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("m", [1, 2, 4, 8, 64, 256])
def test_srht_of_identity_is_scaled_hadamard(orc, m):
    Y = orc.srht(np.eye(m), np.ones(m, np.int8), np.arange(m, dtype=np.int32))
    assert np.abs(Y * np.sqrt(m) - scipy.linalg.hadamard(m)).max() <= 1e-14


@pytest.mark.parametrize("d", [4, 16, 64, 256, 1024])
def test_srht_matches_radix4_fwht(orc, d):
    rng = np.random.default_rng(d)
    x = rng.standard_normal(d)
    dsign = rng.choice(np.array([-1, 1], np.int8), size=d)
    r = rng.integers(0, d, size=17).astype(np.int32)
    ref = fwht_rad4(dsign * x)[r] / np.sqrt(r.shape[0])
    assert rel(orc.srht(x.reshape(-1, 1), dsign, r)[:, 0], ref) <= 1e-13


def test_srht_all_rows_is_orthogonal(orc):
    rng = np.random.default_rng(1)
    m, n = 512, 6
    X = rng.standard_normal((m, n))
    dsign = rng.choice(np.array([-1, 1], np.int8), size=m)
    Y = orc.srht(X, dsign, np.arange(m, dtype=np.int32))
    # k = m, every row once: S = m^{-1/2} H D is orthogonal
    assert rel(Y.T @ Y, X.T @ X) <= 1e-13


def test_srht_zero_padding_and_sampling(orc):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((5, 3))
    dsign = np.array([1, -1, -1, 1, -1], np.int8)
    r = np.array([7, 3, 3, 0, 5], np.int32)
    Xp = np.vstack([X, np.zeros((3, 3))])
    dp = np.concatenate([dsign, np.ones(3, np.int8)])
    Y = orc.srht(X, dsign, r)
    assert np.array_equal(Y, orc.srht(Xp, dp, r))
    assert np.array_equal(Y[1], Y[2])           # a row sampled twice
    H = scipy.linalg.hadamard(8)
    assert rel(Y, (H[r] @ (dp[:, None] * Xp)) / np.sqrt(5)) <= 1e-15
    with pytest.raises(orc.OracleError):
        orc.srht(X, dsign, np.array([8], np.int32))  # outside [0, m)


def test_srht_norm_in_expectation(orc):
    rng = np.random.default_rng(3)
    m, k = 256, 16
    x = rng.standard_normal((m, 1))
    vals = []
    for t in range(400):
        g = np.random.default_rng(1000 + t)
        dsign = g.choice(np.array([-1, 1], np.int8), size=m)
        r = g.integers(0, m, size=k).astype(np.int32)
        vals.append(float((orc.srht(x, dsign, r) ** 2).sum()))
    vals = np.array(vals)
    nx = float((x ** 2).sum())
    assert abs(vals.mean() - nx) <= 5 * vals.std() / np.sqrt(len(vals))


def test_count_srht_lstsq_orthogonal_sketch_is_exact(orc):
    # C = I (k1 = d, identity buckets, + signs) and every SRHT row once:
    # S is orthogonal, so sketch-and-solve is the least-squares solution
    rng = np.random.default_rng(4)
    d, n = 256, 5
    A = rng.standard_normal((d, n))
    B = A @ rng.standard_normal((n, 2)) + 0.1 * rng.standard_normal((d, 2))
    h = np.arange(d, dtype=np.int32)
    s = np.ones(d, np.int8)
    dsign = rng.choice(np.array([-1, 1], np.int8), size=d)
    X = orc.count_srht_lstsq(A, B, h, s, d, dsign, np.arange(d, dtype=np.int32))
    Xl = np.linalg.lstsq(A, B, rcond=None)[0]
    assert rel(X, Xl) <= 1e-12
