"""Pins of the oracle's FP16 Gaussian-stage reference: FP16 rounding of FP32
values and the per-column power-of-two scale of the FP16 stage.

The rounding is checked against a brute-force nearest search over the table
of every finite binary16 value, decoded here from its bit fields (sign,
5-bit exponent with bias 15, 10-bit fraction; subnormals at exponent field
0), ties going to the pattern with an even fraction; and against NumPy's own
float32 -> float16 conversion.  The column scale is checked against its
definition (largest scaled magnitude in [2^14, 2^15)), against exact round
trips of FP16-representable columns, and through the composite solve, which
must not change when every scaled value is already an FP16 number.
"""
import bisect
import math

import numpy as np
import pytest

import synth


def _f16_table():
    """(values, patterns) of every finite non-negative binary16 number,
    ascending, decoded from the bit fields."""
    vals, pats = [], []
    for e in range(31):          # exponent field 31 is infinity / NaN
        for f in range(1024):
            if e == 0:
                v = math.ldexp(f, -24)                  # 2^-14 * f / 1024
            else:
                v = math.ldexp(1024 + f, e - 25)        # 2^(e-15) * (1 + f / 1024)
            vals.append(v)
            pats.append((e << 10) | f)
    return vals, pats


_VALS, _PATS = _f16_table()


def _round_f16_brute(x: float) -> float:
    if math.isnan(x) or math.isinf(x):
        return x
    a = abs(x)
    if a >= 65520.0:            # halfway to 2^16 and beyond: overflow
        r = math.inf
    else:
        j = bisect.bisect_left(_VALS, a)
        if j == len(_VALS):      # above 65504, below the overflow threshold
            r = _VALS[-1]
        elif _VALS[j] == a:
            r = a
        else:
            lo, hi = _VALS[j - 1], _VALS[j]
            if a - lo < hi - a:
                r = lo
            elif hi - a < a - lo:
                r = hi
            else:                # tie: the even fraction
                r = lo if (_PATS[j - 1] & 1) == 0 else hi
    return -r if math.copysign(1.0, x) < 0 else r


def _edge_values():
    v = [0.0, -0.0, 1.0, -1.0, 65504.0, 65505.0, 65519.0, 65519.996, 65520.0, 70000.0,
         -65520.0, 2.0 ** -14, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -25, 2.0 ** -26,
         5 * 2.0 ** -26, 2.0 ** -15 + 2.0 ** -25, 1.0e-30, 3.0e38]
    # exact ties between neighbouring binary16 numbers at several binades
    for e in (-20, -14, -13, -1, 0, 5, 14, 15):
        for f in (0, 1, 2, 3, 1022, 1023):
            base = math.ldexp(1024 + f, e - 10)
            v.append(base + math.ldexp(1.0, e - 11))      # halfway up
            v.append(-(base + math.ldexp(1.0, e - 11)))
    return np.array(v, dtype=np.float32)


def test_round_f16_brute_force(orc):
    rng = np.random.default_rng(16)
    x = np.concatenate([
        _edge_values(),
        (rng.standard_normal(3000) * np.exp2(rng.integers(-30, 18, 3000))).astype(np.float32),
        rng.uniform(-65536, 65536, 500).astype(np.float32),
    ])
    got = orc.round_f16(x)
    want = np.array([_round_f16_brute(float(t)) for t in x], dtype=np.float32)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert np.all(same), x[~same][:5]
    # signed zeros keep their sign
    assert np.array_equal(np.signbit(got[want == 0]), np.signbit(want[want == 0]))


def test_round_f16_matches_numpy_cast(orc):
    rng = np.random.default_rng(17)
    x = np.concatenate([
        _edge_values(),
        (rng.standard_normal(20000) * np.exp2(rng.integers(-28, 17, 20000))).astype(np.float32),
        np.array([np.nan, np.inf, -np.inf], dtype=np.float32),
    ])
    got = orc.round_f16(x)
    with np.errstate(over="ignore"):
        want = x.astype(np.float16).astype(np.float32)
    assert np.all((got == want) | (np.isnan(got) & np.isnan(want)))


def test_f16_col_exp_definition(orc):
    for m in (1.0, 1.5, 2.0 ** 14, 2.0 ** 15, 3.0e4, 7.25e-3, 2.0 ** -20, 123456.0):
        y = np.array([0.25 * m, -m, 0.5 * m], dtype=np.float32)
        e = orc.f16_col_exp(y)
        assert e == math.floor(math.log2(float(np.float32(m)))) - 14
        scaled = float(np.float32(m)) * 2.0 ** -e
        assert 2.0 ** 14 <= scaled < 2.0 ** 15
    assert orc.f16_col_exp(np.zeros(5, np.float32)) == 0
    assert orc.f16_col_exp(np.array([1.0, np.nan], np.float32)) == 0
    assert orc.f16_col_exp(np.array([np.inf, 1.0], np.float32)) == 0
    assert orc.f16_col_exp(np.array([3.0e38], np.float32)) == 112          # clamped
    assert orc.f16_col_exp(np.array([1.0e-40], np.float32)) == -112        # clamped


def test_round_f16_colscaled_exact_and_bounded(orc):
    rng = np.random.default_rng(18)
    k = 4000
    # columns of FP16-representable values times 2^p: unchanged
    cols = []
    for p in (-30, -3, 0, 9, 40):
        ints = rng.integers(-2047, 2048, k).astype(np.float64)
        ints[7] = 2047.0
        cols.append(ints * 2.0 ** p)
    Y = np.asarray(np.stack(cols, axis=1), dtype=np.float32, order="F")
    assert np.array_equal(orc.round_f16_colscaled(Y), Y.astype(np.float64))
    # general columns of very different scales: each scaled value is rounded
    # once, so |error| <= 2^-11 |y| in FP16's normal range and <= 2^-25 (times
    # the column's scale) below it
    Y = np.asarray(rng.standard_normal((k, 4)) * np.array([1e-12, 1.0, 3e3, 1e20]),
                   dtype=np.float32, order="F")
    Y[5, 1] = 1e-9   # far below the column's largest magnitude: FP16 subnormal after scaling
    R = orc.round_f16_colscaled(Y)
    for c in range(Y.shape[1]):
        e = orc.f16_col_exp(Y[:, c])
        y = Y[:, c].astype(np.float64)
        err = np.abs(R[:, c] - y)
        normal = np.abs(y) * 2.0 ** -e >= 2.0 ** -14
        assert np.all(err[normal] <= 2.0 ** -11 * np.abs(y[normal]))
        assert np.all(err[~normal] <= 2.0 ** (e - 25))
        assert 2.0 ** 14 <= np.max(np.abs(y)) * 2.0 ** -e < 2.0 ** 15
    # a zero column stays zero
    assert np.all(orc.round_f16_colscaled(np.zeros((10, 1), np.float32)) == 0.0)


def test_composite_f16_exact_when_representable(orc):
    # small-integer data: every sketch entry is a small integer, so the
    # scaled sketch is exactly representable in FP16 and the FP16 path must
    # reproduce the unrounded FP32 path bit for bit
    rng = np.random.default_rng(19)
    d, n, nrhs, k, k2 = 3000, 4, 2, 64, 16
    A = np.asfortranarray(rng.integers(-3, 4, (d, n)).astype(np.float32))
    B = np.asfortranarray(rng.integers(-3, 4, (d, nrhs)).astype(np.float32))
    h = synth.bucket_map(d, k, seed=19)
    s = synth.signs(d, seed=19)
    G = synth.gaussian_sketch(k2, k, seed=19, dtype="f64")
    X0, Y0, Z0 = orc.sketch_lstsq(A, B, h, s, G, k)
    X1, Y1, Z1 = orc.sketch_lstsq(A, B, h, s, G, k, y_f16=True)
    assert np.array_equal(Y0, Y1)
    assert np.array_equal(Z0, Z1) and np.array_equal(X0, X1)
    # and with data that is not representable the rounding does act
    Af = np.asfortranarray(rng.standard_normal((d, n)).astype(np.float32))
    Bf = np.asfortranarray(rng.standard_normal((d, nrhs)).astype(np.float32))
    _, _, Za = orc.sketch_lstsq(Af, Bf, h, s, G, k)
    _, Yb, Zb = orc.sketch_lstsq(Af, Bf, h, s, G, k, y_f16=True)
    assert not np.array_equal(Za, Zb)
    Zr = orc.gemm(G, orc.round_f16_colscaled(Yb))
    assert np.array_equal(Zb, Zr)
