"""GPU parity of the normal-equations least-squares solver (Sec. 6.3: Gram
matrix, Cholesky, two triangular solves) against the oracle, through the C
ABI.

Bar: FP64 normwise relative 1e-12 against the oracle on the same inputs for
kappa(A) <= 10.  The normal equations' forward error grows like
kappa(A)^2 u (the Gram matrix squares the condition number), and the device
and the oracle sum the Gram matrix in different orders, so at kappa = 1e2
the two may differ by about n kappa^2 u = 64 * 1e4 * 1.1e-16 = 7e-11: the bar
there is 1e-10.  FP32 data: the same bars against the oracle on the
promoted data.  At the full 4,194,304 x 64 size the least-squares optimality
A^T (B - A X) = 0 is checked instead, and agreement with rand_cholQR.
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


def _problem(d, n, nrhs, kappa, seed, dtype=np.float64, noise=1e-2):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d, n)) * np.logspace(0, -np.log10(kappa), n)
    B = A @ rng.standard_normal((n, nrhs)) + noise * rng.standard_normal((d, nrhs))
    return np.asfortranarray(A, dtype=dtype), np.asfortranarray(B, dtype=dtype)


# (d, n, nrhs, kappa): ragged d (not a multiple of 4 or 16); the column
# layouts n + nrhs <= 16 NTI, n + nrhs = 16 NTI + 1 (one spare column, vector
# path) and n + nrhs > 16 NTI + 1 (one more matrix-core tile)
CASES = [(1000, 3, 1, 1.0), (12345, 8, 2, 10.0), (65537, 16, 3, 10.0), (100003, 33, 1, 10.0),
         (200003, 64, 1, 10.0), (5000, 60, 16, 10.0), (4099, 64, 2, 1.0), (7777, 48, 1, 10.0),
         (30001, 20, 12, 10.0), (17, 5, 1, 1.0), (10, 3, 2, 1.0)]


@pytest.mark.parametrize("d,n,nrhs,kappa", CASES)
def test_normal_equations_fp64_parity(ms, orc, d, n, nrhs, kappa):
    print("normal_equations f64 d=%d n=%d nrhs=%d kappa=%g" % (d, n, nrhs, kappa), flush=True)
    A, B = _problem(d, n, nrhs, kappa, seed=d + n)
    R = ms.empty_colmajor(n, n, torch.float64, "cuda")
    X, _, ws = ms.normal_equations_lstsq(to_dev(A), to_dev(B), R=R)
    ms.check_status(ws)
    Xr = orc.normal_equations(A, B)
    assert rel(to_host(X), Xr) <= 1e-12
    Rg = to_host(R)
    assert np.all(np.tril(Rg, -1) == 0.0) and np.all(np.diag(Rg) > 0.0)
    assert rel(Rg.T @ Rg, A.T @ A) <= 1e-13


def test_normal_equations_kappa_1e2(ms, orc):
    A, B = _problem(100003, 64, 2, 1e2, seed=9)
    X, _, ws = ms.normal_equations_lstsq(to_dev(A), to_dev(B))
    ms.check_status(ws)
    assert rel(to_host(X), orc.normal_equations(A, B)) <= 1e-10


@pytest.mark.parametrize("n,nrhs", [(16, 2), (64, 1)])
def test_normal_equations_fp32(ms, orc, n, nrhs):
    A, B = _problem(70001, n, nrhs, 10.0, seed=7, dtype=np.float32)
    X, _, ws = ms.normal_equations_lstsq(to_dev(A), to_dev(B))
    ms.check_status(ws)
    Xr = orc.normal_equations(A.astype(np.float64), B.astype(np.float64))
    assert rel(to_host(X), Xr) <= 1e-12


def test_normal_equations_repeatable(ms):
    # fixed summation order: two calls give the same bits
    A, B = _problem(123457, 40, 3, 10.0, seed=4)
    Ad, Bd = to_dev(A), to_dev(B)
    X1, _, ws = ms.normal_equations_lstsq(Ad, Bd)
    X2, _, _ = ms.normal_equations_lstsq(Ad, Bd, ws=ws)
    ms.check_status(ws)
    assert torch.equal(X1, X2)


def test_normal_equations_full_size(ms):
    # the 4,194,304 x 64 FP64 workload: A^T (B - A X) = 0 up to rounding,
    # and the same optimum as rand_cholQR
    d, n, k, k2 = 4194304, 64, 8192, 128
    g = torch.Generator(device="cuda")
    g.manual_seed(14209)
    A = torch.randn((n, d), generator=g, device="cuda", dtype=torch.float64).t()
    xs = torch.randn((n, 1), generator=g, device="cuda", dtype=torch.float64)
    B = ms.empty_colmajor(d, 1, torch.float64, "cuda")
    B.copy_(A @ xs + 1e-2 * torch.randn((d, 1), generator=g, device="cuda", dtype=torch.float64))
    X, _, ws = ms.normal_equations_lstsq(A, B)
    ms.check_status(ws)
    r = B - A @ X
    grad = (A.t() @ r).norm().item()
    scale = (A.norm() * r.norm()).item()
    assert grad / scale <= 1e-13, grad / scale
    h = torch.randint(0, k, (d,), generator=g, device="cuda", dtype=torch.int32)
    s = (torch.randint(0, 2, (d,), generator=g, device="cuda", dtype=torch.int8) * 2 - 1)
    G = ms.empty_colmajor(k2, k, torch.float64, "cuda")
    G.copy_(torch.randn((k, k2), generator=g, device="cuda", dtype=torch.float64).t() / np.sqrt(k2))
    Xq, _, wq = ms.rand_cholqr_lstsq(A, B, h, s, G, k)
    ms.check_status(wq)
    assert rel(to_host(X), to_host(Xq)) <= 1e-12


# Wide problems (n > 64, up to 256 columns and 16 right-hand sides): the
# tiled Gram pass and the blocked Cholesky.  Ragged shapes: a partial last
# 64-column block, n + nrhs not a multiple of 16, d not a multiple of 16,
# d barely above n.  Bar: the two sides sum the Gram matrix in different
# orders, and the normal equations amplify such differences by kappa(A)^2,
# so X agrees to about n kappa(A)^2 u (times a small factor); never looser
# than the FP64 bar of 1e-12 where that product is below 1e-13.
WIDE_CASES = [(20011, 65, 1, 10.0), (50000, 100, 3, 10.0), (100003, 128, 1, 10.0),
              (30000, 200, 16, 10.0), (70001, 256, 16, 10.0), (400, 256, 1, 1.0),
              (65536, 250, 7, 1.0)]


@pytest.mark.parametrize("d,n,nrhs,kappa", WIDE_CASES)
def test_normal_equations_wide_parity(ms, orc, d, n, nrhs, kappa):
    print("normal_equations wide d=%d n=%d nrhs=%d kappa=%g" % (d, n, nrhs, kappa), flush=True)
    A, B = _problem(d, n, nrhs, kappa, seed=d + n)
    R = ms.empty_colmajor(n, n, torch.float64, "cuda")
    X, _, ws = ms.normal_equations_lstsq(to_dev(A), to_dev(B), R=R)
    ms.check_status(ws)
    Xr = orc.normal_equations(A, B)
    ka = np.linalg.cond(A)
    tol = max(1e-12, 10 * n * ka ** 2 * 2.0 ** -53)
    err = rel(to_host(X), Xr)
    print("  kappa(A) %.3g err %.3e tol %.3e" % (ka, err, tol))
    assert err <= tol
    Rg = to_host(R)
    assert np.all(np.tril(Rg, -1) == 0.0) and np.all(np.diag(Rg) > 0.0)
    assert rel(Rg.T @ Rg, A.T @ A) <= 1e-13


def test_normal_equations_wide_fp32_and_singular(ms, orc):
    A, B = _problem(70001, 128, 2, 10.0, seed=8, dtype=np.float32)
    X, _, ws = ms.normal_equations_lstsq(to_dev(A), to_dev(B))
    ms.check_status(ws)
    Xr = orc.normal_equations(A.astype(np.float64), B.astype(np.float64))
    assert rel(to_host(X), Xr) <= 1e-11
    A2, B2 = _problem(5000, 150, 1, 1.0, seed=9)
    A2[:, 130] = 0.0   # breakdown in the third diagonal block
    X2, _, ws2 = ms.normal_equations_lstsq(to_dev(A2), to_dev(B2))
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws2)
    assert e.value.code == ms.MS_ERR_SINGULAR
    assert np.all(np.isnan(to_host(X2)))


def test_normal_equations_errors(ms):
    A, B = _problem(3000, 8, 1, 1.0, seed=5)
    Ad = to_dev(A)
    Ad[:, 3] = 0.0  # rank deficient: the Cholesky factorisation breaks down
    X, _, ws = ms.normal_equations_lstsq(Ad, to_dev(B))
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_SINGULAR
    assert np.all(np.isnan(to_host(X)))
    for n, nrhs in ((257, 1), (8, 17), (260, 16)):
        A2, B2 = _problem(500, n, nrhs, 1.0, seed=6)
        with pytest.raises(ms.MsketchError) as e:
            ms.normal_equations_lstsq(to_dev(A2), to_dev(B2))
        assert e.value.code == ms.MS_ERR_UNSUPPORTED
