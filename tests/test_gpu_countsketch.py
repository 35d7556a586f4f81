"""GPU parity: sketch plan and CountSketch (all three variants) against the
oracle, through the C ABI.

Bar: bit-exact for the plan (integers) and for the deterministic sorted mode;
normwise relative 1e-12 (FP64) / 1e-5 (FP32) for the atomic and LDS modes,
whose association order differs from the sequential fold.
"""
import os

import numpy as np
import pytest

import synth
from gpu_util import bits_equal, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "canonical_fold.txt")


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


def _inputs(d, n, k, seed, dtype=np.float64):
    A = synth.normal_matrix(d, n, seed=seed, dtype=dtype)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    return A, h, s


# ------------------------------------------------------------------- plan
@pytest.mark.parametrize("d,k", [(1, 1), (777, 7), (65536, 2048), (300000, 40), (4194304, 8192)])
def test_bucket_plan_bit_exact(ms, orc, d, k):
    print("plan d=%d k=%d" % (d, k), flush=True)
    h = synth.bucket_map(d, k, seed=d % 97)
    cnt, off, perm, ws = ms.bucket_plan(to_dev(h), k)
    ms.check_status(ws)
    off_ref, perm_ref = orc.bucket_plan(h, k)
    assert np.array_equal(to_host(cnt).astype(np.int64), orc.bucket_hist(h, k))
    assert np.array_equal(to_host(off).astype(np.int64), off_ref)
    assert np.array_equal(to_host(perm).astype(np.int64), perm_ref)


def test_bucket_plan_long_bucket_blocked(ms, orc):
    # up to MS_SORTED_BLOCKED_MAX_K buckets the plan is a blocked stable
    # counting sort: a bucket holding most rows is planned exactly
    d, k = 3 * ms.MS_SORTED_MAX_SEGMENT + 5, 2
    h = np.zeros(d, np.int32)
    h[::7] = 1
    cnt, off, perm, ws = ms.bucket_plan(to_dev(h), k)
    ms.check_status(ws)
    off_ref, perm_ref = orc.bucket_plan(h, k)
    assert np.array_equal(to_host(off).astype(np.int64), off_ref)
    assert np.array_equal(to_host(perm).astype(np.int64), perm_ref)


def test_bucket_plan_segment_limit_reported(ms):
    # beyond MS_SORTED_BLOCKED_MAX_K buckets each bucket is sorted in LDS: one
    # longer than the limit is reported, not mis-sorted
    k = ms.MS_SORTED_BLOCKED_MAX_K + 1
    d = 3 * ms.MS_SORTED_MAX_SEGMENT
    h = (np.arange(d, dtype=np.int64) % k).astype(np.int32)
    h[::2] = 0
    cnt, off, perm, ws = ms.bucket_plan(to_dev(h), k)
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_UNSUPPORTED


# ------------------------------------------------------------------- CountSketch
CASES = [
    # d, n, k, dtype
    (1, 1, 1, np.float64),
    (1000, 3, 64, np.float64),
    (12345, 5, 300, np.float64),   # ragged: k not a power of two, d % 4 != 0
    (65536, 32, 2048, np.float64),  # the 65,536 x 32 FP64, k = 2048 workload
    (12347, 7, 301, np.float32),
    (200000, 9, 4096, np.float32),
    (300, 4, 2000, np.float64),    # k > d: most buckets empty
]


@pytest.mark.parametrize("mode", ["sorted", "lds", "atomic"])
@pytest.mark.parametrize("d,n,k,dtype", CASES)
def test_countsketch_parity(ms, orc, mode, d, n, k, dtype):
    print("countsketch mode=%s d=%d n=%d k=%d %s" % (mode, d, n, k, np.dtype(dtype)), flush=True)
    A, h, s = _inputs(d, n, k, seed=d + n + k, dtype=dtype)
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(s), k, mode=mode)
    ms.check_status(ws)
    Yg = to_host(Y)
    Yr = orc.countsketch(A, h, s, k)
    assert Yg.shape == (k, n) and Yg.dtype == dtype
    if mode == "sorted":
        assert bits_equal(Yg, Yr)
    else:
        assert rel(Yg, Yr) <= (1e-12 if dtype == np.float64 else 1e-5)


@pytest.mark.parametrize("mode", ["sorted", "lds"])
def test_countsketch_full_c2_shape(ms, orc, mode):
    # A 4,194,304 x 65 FP64 ([A | b] of the multisketch least-squares workload), k = 8192
    d, n, k = 4194304, 65, 8192
    print("countsketch full d=%d n=%d k=%d mode=%s" % (d, n, k, mode), flush=True)
    A, h, s = _inputs(d, n, k, seed=14209)
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(s), k, mode=mode)
    ms.check_status(ws)
    Yr = orc.countsketch(A, h, s, k)
    if mode == "sorted":
        assert bits_equal(to_host(Y), Yr)
    else:
        assert rel(to_host(Y), Yr) <= 1e-12


@pytest.mark.parametrize("dtype,k", [(np.float64, 32768), (np.float32, 65536), (np.float32, 131072)])
def test_countsketch_bucket_tiles(ms, orc, dtype, k):
    # more buckets than one workgroup's LDS holds: bucket tiles
    d, n = 1 << 20, 3
    print("countsketch tiles k=%d %s" % (k, np.dtype(dtype)), flush=True)
    A, h, s = _inputs(d, n, k, seed=5, dtype=dtype)
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(s), k, mode="lds")
    ms.check_status(ws)
    assert rel(to_host(Y), orc.countsketch(A, h, s, k)) <= (1e-12 if dtype == np.float64 else 1e-5)


@pytest.mark.parametrize("d,n,k,dtype,tiled", [(300001, 20, 65536, np.float32, True),
                                               (1000, 8, 131072, np.float32, True),
                                               (8192 * 3 + 5, 3, 70001, np.float64, True),
                                               (50000, 2, 41000, np.float32, True),
                                               (8192, 1, 61441, np.float64, True),
                                               (200000, 32, 32768, np.float64, False),
                                               (8192 * 3 + 5, 3, 40000, np.float64, False),
                                               (8192, 1, 16385, np.float64, False)])
def test_countsketch_tiled_plan(ms, orc, d, n, k, dtype, tiled):
    # more buckets than one workgroup's LDS holds (k > 16384).  From four
    # bucket tiles up (k > 40960) the rows of each 8192-row block are grouped
    # by bucket tile first and each tile's workgroups visit only their rows;
    # with two tiles every tile's workgroups stream all rows (untiled).
    # Ragged shapes: a partial last block, one block only, bucket counts that
    # are not powers of two, tiles of unequal length.  With the plan the
    # workspace holds it (4 bytes per row, block padded) besides the codes.
    a_dt = ms.MS_F64 if dtype == np.float64 else ms.MS_F32
    nblk = (d + 8191) // 8192
    extra = (ms.workspace_size("countsketch", d=d, n=n, k=k, a_dtype=a_dt, mode="lds")
             - ms.workspace_size("countsketch", d=d, n=n, k=k, a_dtype=a_dt, mode="atomic"))
    if tiled:
        assert extra >= nblk * 8192 * 4
    print("countsketch tiled d=%d n=%d k=%d %s" % (d, n, k, np.dtype(dtype)), flush=True)
    A, h, s = _inputs(d, n, k, seed=9, dtype=dtype)
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(s), k, mode="lds")
    ms.check_status(ws)
    assert rel(to_host(Y), orc.countsketch(A, h, s, k)) <= (1e-12 if dtype == np.float64 else 1e-5)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_countsketch_tiled_accumulate_row_blocks(ms, orc, dtype):
    # Y += C A over two row blocks (the streaming form of Sec. 7) through the
    # packed codes, with the tiled plan built from the codes in the workspace
    import torch
    d, n, k, split = 150001, 5, 65536, 70001
    a_dt = ms.MS_F64 if dtype == np.float64 else ms.MS_F32
    A, h, s = _inputs(d, n, k, seed=19, dtype=dtype)
    Y = ms.empty_colmajor(k, n, torch.float64 if dtype == np.float64 else torch.float32, "cuda")
    Y.zero_()
    for r0, r1 in ((0, split), (split, d)):
        print("accumulate rows %d..%d" % (r0, r1), flush=True)
        code, _ = ms.pack_sketch(to_dev(h[r0:r1]), to_dev(s[r0:r1]), k)
        ws = ms.workspace(ms.workspace_size("countsketch", d=r1 - r0, n=n, k=k, a_dtype=a_dt), "cuda")
        ms.countsketch_accumulate(to_dev(A[r0:r1]), code, k, Y, mode="lds", ws=ws)
        ms.check_status(ws)
    assert rel(to_host(Y), orc.countsketch(A, h, s, k)) <= (1e-12 if dtype == np.float64 else 1e-5)


def test_countsketch_tiled_range_errors(ms):
    d, n, k = 20000, 2, 32768
    A, h, s = _inputs(d, n, k, seed=3)
    hb = h.copy()
    hb[12345] = k
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(hb), to_dev(s), k, mode="lds")
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE
    sb = s.copy()
    sb[9000] = 0
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(sb), k, mode="lds")
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE


@pytest.mark.parametrize("mode", ["sorted", "lds", "atomic"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("off", [0, 1])
def test_countsketch_strided_lda(ms, orc, mode, dtype, off):
    # leading dimension not a multiple of the vector width, and (off = 1) a
    # first column that starts one element past an aligned address: the
    # vector loads are element-aligned only
    d, n, k = 5001, 3, 128
    print("strided mode=%s %s off=%d" % (mode, np.dtype(dtype), off), flush=True)
    A, h, s = _inputs(d, n, k, seed=9, dtype=dtype)
    big = np.zeros((d + 3, n), dtype=dtype)
    big[off:off + d] = A
    At = to_dev(big)[off:off + d]
    assert At.stride(1) == d + 3
    Y, ws = ms.countsketch_apply(At, to_dev(h), to_dev(s), k, mode=mode)
    ms.check_status(ws)
    Yr = orc.countsketch(A, h, s, k)
    if mode == "sorted":
        assert bits_equal(to_host(Y), Yr)
    else:
        assert rel(to_host(Y), Yr) <= (1e-12 if dtype == np.float64 else 1e-5)


def _golden_cases():
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            dt, vals, expect = [t.strip() for t in line.split(";")]
            yield dt, [float(v) for v in vals.split(",")], float(expect)


@pytest.mark.parametrize("case", list(_golden_cases()))
def test_sorted_mode_reproduces_canonical_fold(ms, case):
    dt, vals, expect = case
    dtype = np.float64 if dt == "f64" else np.float32
    d = 3 * len(vals)
    A = np.ones((d, 1), dtype=dtype)
    h = np.ones(d, np.int32)
    s = np.ones(d, np.int8)
    for j, v in enumerate(vals):
        i = 3 * j + 1
        h[i] = 0
        A[i, 0], s[i] = (-v, -1) if j % 2 else (v, 1)
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(s), 2, mode="sorted")
    ms.check_status(ws)
    got = float(to_host(Y)[0, 0])
    assert got == expect and np.signbit(got) == np.signbit(expect)


def test_empty_rows_and_columns(ms):
    import torch
    k = 16
    Y, ws = ms.countsketch_apply(ms.empty_colmajor(0, 3, torch.float64),
                                 torch.empty(0, dtype=torch.int32, device="cuda"),
                                 torch.empty(0, dtype=torch.int8, device="cuda"), k)
    ms.check_status(ws)
    assert np.array_equal(to_host(Y), np.zeros((k, 3)))
    Y, ws = ms.countsketch_apply(ms.empty_colmajor(10, 0, torch.float64),
                                 to_dev(np.zeros(10, np.int32)), to_dev(np.ones(10, np.int8)), k)
    ms.check_status(ws)
    assert Y.shape == (k, 0)


@pytest.mark.parametrize("mode", ["sorted", "lds", "atomic"])
def test_range_errors_reported(ms, mode):
    d, n, k = 100, 2, 8
    A, h, s = _inputs(d, n, k, seed=1)
    hb = h.copy()
    hb[37] = k
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(hb), to_dev(s), k, mode=mode)
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE
    sb = s.copy()
    sb[5] = 0
    Y, ws = ms.countsketch_apply(to_dev(A), to_dev(h), to_dev(sb), k, mode=mode)
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE
