"""GPU parity of the hash-generated CountSketch (Sec. 8's future-work variant:
each row's bucket and sign computed from (seed, row), no stored h and s)
against the oracle, through the C ABI.

Bars: the generated h and s are integers and must match the oracle's bit for
bit; the sketch Y is compared normwise at 1e-12 (FP64) and 1e-5 (FP32), the
CountSketch bars (the LDS accumulation order differs from the oracle's
ascending fold).
"""
import numpy as np
import pytest
import torch

from gpu_util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


@pytest.mark.parametrize("d,k,seed", [(1, 1, 0), (1000, 1, 5), (4097, 128, 14209),
                                      (100003, 2048, 2**64 - 1), (65536, (1 << 31) - 2, 77),
                                      (333333, 1 << 20, 123456789)])
def test_hash_sketch_bit_exact(ms, orc, d, k, seed):
    print("hash_sketch d=%d k=%d seed=%d" % (d, k, seed), flush=True)
    h, s = ms.hash_sketch(d, k, seed)
    hr, sr = orc.hash_sketch(d, k, seed)
    assert np.array_equal(to_host(h), hr)
    assert np.array_equal(to_host(s), sr)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("d,n,k", [(1000, 1, 7), (65537, 8, 128), (100003, 33, 2048),
                                   (20011, 3, 40000), (4096, 65, 8192)])
def test_countsketch_hashed_parity(ms, orc, dtype, d, n, k):
    print("countsketch_hashed d=%d n=%d k=%d %s" % (d, n, k, np.dtype(dtype).name), flush=True)
    rng = np.random.default_rng(d + n)
    A = np.asfortranarray(rng.standard_normal((d, n)).astype(dtype))
    seed = 1000 + d
    Y, ws = ms.countsketch_hashed(to_dev(A), k, seed)
    ms.check_status(ws)
    Yr = orc.countsketch_hashed(A, k, seed, acc="f64" if dtype == np.float32 else None)
    assert rel(to_host(Y), Yr) <= (1e-12 if dtype == np.float64 else 1e-5)


def test_hashed_equals_stored_vectors(ms):
    # the same sketch through countsketch_apply with the materialised h and s
    d, n, k, seed = 300007, 16, 512, 99
    A = torch.randn((n, d), dtype=torch.float64, device="cuda").t()
    Yh, ws = ms.countsketch_hashed(A, k, seed)
    h, s = ms.hash_sketch(d, k, seed)
    Ys, ws2 = ms.countsketch_apply(A, h, s, k, mode="lds")
    ms.check_status(ws)
    ms.check_status(ws2)
    assert rel(to_host(Yh), to_host(Ys)) <= 1e-12


def test_hashed_full_size_fp32(ms, orc):
    # the narrow workload where stored h and s are 5 of 37 bytes per row
    d, n, k, seed = 1 << 24, 8, 128, 14209
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randn((n, d), generator=g, device="cuda", dtype=torch.float32).t()
    Y, ws = ms.countsketch_hashed(A, k, seed)
    ms.check_status(ws)
    Yr = orc.countsketch_hashed(to_host(A), k, seed, acc="f64")
    assert rel(to_host(Y), Yr) <= 1e-5


def test_countsketch_hashed_empty(ms):
    # no rows: Y is all zero; no columns: nothing to do
    A = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    Y, ws = ms.countsketch_hashed(A, 16, 5)
    ms.check_status(ws)
    assert torch.count_nonzero(Y).item() == 0
    A = torch.zeros((100, 0), dtype=torch.float64, device="cuda")
    Y, ws = ms.countsketch_hashed(A, 16, 5)
    ms.check_status(ws)
    assert Y.shape == (16, 0)


def test_hash_sketch_k_limit(ms):
    # k <= 2^31 - 2, as for every entry point (bucket field 0x7fffffff marks
    # an invalid row)
    with pytest.raises(ms.MsketchError) as e:
        ms.hash_sketch(10, (1 << 31) - 1, 1)
    assert e.value.code == ms.MS_ERR_ARG


def test_hashed_unsupported_modes(ms):
    A = torch.randn((8, 1000), dtype=torch.float64, device="cuda").t()
    for mode, sched in (("sorted", 0), ("atomic", 0), ("auto", 1)):
        o = ms._opts(mode, 0, 0, sched)
        need = ms.workspace_size("countsketch_hashed", d=1000, n=8, k=64)
        ws = ms.workspace(need)
        wp, have = ms._ws_ptr(ws, need)
        Y = ms.empty_colmajor(64, 8, torch.float64, "cuda")
        Ap, lda = ms.colmajor(A, "A")
        Yp, ldy = ms.colmajor(Y, "Y")
        rc = ms._lib.countsketch_hashed(1000, 8, 64, 5, ms.MS_F64, Ap, lda, Yp, ldy,
                                        ms.ctypes.byref(o), wp, have, ms._stream(None))
        assert rc == ms.MS_ERR_UNSUPPORTED
