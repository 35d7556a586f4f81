"""GPU parity of the SRHT (Sec. 5) and of sketch-and-solve with the Count +
SRHT multisketch (Sec. 8's future-work variant) against the oracle, through
the C ABI.

Bar: FP64 normwise relative 1e-12 (the oracle sums each output exactly in
long double; the device's butterflies are within log2(m) u of it).  FP32
input is promoted exactly, so the same bar holds.  At the full 4,194,304 x
64 size (the oracle costs O(d) per output) sampled outputs are checked.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


def _srht_inputs(m, nc, k, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    X = np.asfortranarray(rng.standard_normal((m, nc)).astype(dtype))
    mp = 1 << int(np.ceil(np.log2(m))) if m > 1 else 1
    dsign = rng.choice(np.array([-1, 1], np.int8), size=m)
    r = rng.integers(0, mp, size=k).astype(np.int32)
    return X, dsign, r


# m: a single element, non powers of two (zero padding), the LDS-only sizes,
# exactly one 8192-row block, several blocks with a ragged last one
@pytest.mark.parametrize("m,nc,k", [(1, 1, 1), (7, 3, 5), (1000, 2, 16), (4096, 1, 300),
                                    (8192, 5, 128), (8193, 2, 64), (65536, 3, 17),
                                    (100000, 4, 128), (262144, 65, 256)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_srht_parity(ms, orc, m, nc, k, dtype):
    print("srht m=%d nc=%d k=%d %s" % (m, nc, k, np.dtype(dtype).name), flush=True)
    X, dsign, r = _srht_inputs(m, nc, k, seed=m + nc, dtype=dtype)
    Y, ws = ms.srht_apply(to_dev(X), to_dev(dsign), to_dev(r))
    ms.check_status(ws)
    Yr = orc.srht(X.astype(np.float64), dsign, r)
    assert rel(to_host(Y), Yr) <= 1e-12


def test_srht_many_sampled_rows(ms, orc):
    # k above the 1024 sampled rows kept in LDS: the indices are read from memory
    X, dsign, r = _srht_inputs(40000, 3, 1500, seed=11)
    Y, ws = ms.srht_apply(to_dev(X), to_dev(dsign), to_dev(r))
    ms.check_status(ws)
    assert rel(to_host(Y), orc.srht(X, dsign, r)) <= 1e-12


def test_srht_no_columns(ms):
    X = torch.zeros((1000, 0), dtype=torch.float64, device="cuda")
    dsign = torch.ones(1000, dtype=torch.int8, device="cuda")
    r = torch.zeros(4, dtype=torch.int32, device="cuda")
    Y, ws = ms.srht_apply(X, dsign, r)
    ms.check_status(ws)
    assert Y.shape == (4, 0)


def test_srht_repeatable(ms):
    X, dsign, r = _srht_inputs(300000, 6, 100, seed=5)
    Xd, dd, rd = to_dev(X), to_dev(dsign), to_dev(r)
    Y1, ws = ms.srht_apply(Xd, dd, rd)
    Y2, _ = ms.srht_apply(Xd, dd, rd, ws=ws)
    ms.check_status(ws)
    assert torch.equal(Y1, Y2)


def test_srht_full_size_sampled(ms, orc):
    # A 4,194,304 x 64 FP64 with k = 2n = 128: a few outputs by the oracle
    d, n, k = 4194304, 64, 128
    g = torch.Generator(device="cuda")
    g.manual_seed(14209)
    A = torch.randn((n, d), generator=g, device="cuda", dtype=torch.float64).t()
    dsign = (torch.randint(0, 2, (d,), generator=g, device="cuda", dtype=torch.int8) * 2 - 1)
    r = torch.randint(0, d, (k,), generator=g, device="cuda", dtype=torch.int32)
    Y, ws = ms.srht_apply(A, dsign, r)
    ms.check_status(ws)
    Yh = to_host(Y)
    rh, dh = to_host(r), to_host(dsign)
    for c in (0, 37, 63):
        col = to_host(A[:, c:c + 1].contiguous())
        for j in (0, 77, 127):
            # the oracle's single output, rescaled from 1/sqrt(1) to 1/sqrt(k)
            y = orc.srht(col, dh, rh[j:j + 1])[0, 0] / np.sqrt(k)
            assert abs(Yh[j, c] - y) <= 1e-13 * np.sqrt(d)


def test_srht_range_errors(ms):
    X, dsign, r = _srht_inputs(5000, 2, 8, seed=1)
    r[3] = 8192  # padded m is 8192: outside
    Y, ws = ms.srht_apply(to_dev(X), to_dev(dsign), to_dev(r))
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE
    X, dsign, r = _srht_inputs(20000, 2, 8, seed=2)
    dsign[17] = 0
    Y, ws = ms.srht_apply(to_dev(X), to_dev(dsign), to_dev(r))
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE


def _lstsq_problem(d, n, nrhs, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, n)) * np.logspace(0, -2, n)
    B = A @ rng.standard_normal((n, nrhs)) + 1e-2 * rng.standard_normal((d, nrhs))
    k1, k2 = 2 * n * n, 2 * n
    h = synth.bucket_map(d, k1, seed=seed)
    s = synth.signs(d, seed=seed)
    m1 = 1 << int(np.ceil(np.log2(k1)))
    dsign = rng.choice(np.array([-1, 1], np.int8), size=k1)
    r = rng.integers(0, m1, size=k2).astype(np.int32)
    return (np.asfortranarray(A.astype(dtype)), np.asfortranarray(B.astype(dtype)), h, s, k1,
            dsign, r)


# n = 66: k1 = 2 n^2 = 8712 rows, so the second stage spans two 8192-row blocks
@pytest.mark.parametrize("d,n,nrhs", [(5000, 4, 1), (65537, 16, 2), (200003, 64, 1),
                                      (100000, 33, 3), (60000, 66, 1)])
def test_count_srht_lstsq_parity(ms, orc, d, n, nrhs):
    print("count_srht_lstsq d=%d n=%d nrhs=%d" % (d, n, nrhs), flush=True)
    A, B, h, s, k1, dsign, r = _lstsq_problem(d, n, nrhs, seed=d + n)
    X, ws = ms.count_srht_lstsq(to_dev(A), to_dev(B), to_dev(h), to_dev(s), k1, to_dev(dsign),
                                to_dev(r), mode="sorted")
    ms.check_status(ws)
    Xr = orc.count_srht_lstsq(A, B, h, s, k1, dsign, r)
    assert rel(to_host(X), Xr) <= 1e-12
    # the LDS CountSketch (another summation order) at the same bar
    X2, ws2 = ms.count_srht_lstsq(to_dev(A), to_dev(B), to_dev(h), to_dev(s), k1, to_dev(dsign),
                                  to_dev(r), mode="lds")
    ms.check_status(ws2)
    assert rel(to_host(X2), Xr) <= 1e-12


def test_count_srht_lstsq_fp32(ms, orc):
    A, B, h, s, k1, dsign, r = _lstsq_problem(70001, 16, 2, seed=9, dtype=np.float32)
    X, ws = ms.count_srht_lstsq(to_dev(A), to_dev(B), to_dev(h), to_dev(s), k1, to_dev(dsign),
                                to_dev(r), mode="sorted")
    ms.check_status(ws)
    Xr = orc.count_srht_lstsq(A, B, h, s, k1, dsign, r)
    assert rel(to_host(X), Xr) <= 1e-12
