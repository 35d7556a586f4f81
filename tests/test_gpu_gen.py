"""GPU checks of the device request generator (ms_gen_lstsq_request), which
makes the serving workload's inputs: A = Z diag(D) Q with D_j =
kappa^(-j/(n-1)) and Q = H(u1) H(u2), B = A x* + 1e-6 N(0,1), h, s and
G = N(0,1)/sqrt(k2).

What fixes the expected values:
* Q is orthogonal and Z/sqrt(d) has singular values in
  [1 - sqrt(n/d), 1 + sqrt(n/d)] up to a small multiple (Marchenko-Pastur
  edges), so by Ostrowski's bound for Z D the j-th singular value of
  A/sqrt(d) lies within that band around D_j: the prescribed condition number
  (Sec. 6.3's test matrices).
* The reflections mix the columns: A^T A is far from diagonal when kappa > 1.
* B - A x* is the noise: 1e-6 N(0,1) plus the FP32 rounding of the product.
* h is uniform on [0, k) (chi-square over the buckets), s is +-1 with mean 0.
* G's BF16 form is the round-to-nearest-even of its FP32 form and the FP64
  form is the exact promotion (same seed).
* Entries are Gaussian: skewness near 0 and kurtosis near 3.
* Everything is a function of the seed: two calls agree bit for bit.
"""
import numpy as np
import pytest
import torch

from gpu_util import to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


def test_generator_deterministic(ms):
    print("gen determinism d=50000 n=24 nrhs=3", flush=True)
    a = ms.gen_lstsq_request(11, 50000, 24, 3, 1e4, 1152, 48, g_dtype=ms.MS_BF16)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = ms.gen_lstsq_request(11, 50000, 24, 3, 1e4, 1152, 48, g_dtype=ms.MS_BF16, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    for key in ("A", "B", "xstar", "h", "s", "G"):
        assert torch.equal(a[key], b[key]), key
    c = ms.gen_lstsq_request(12, 50000, 24, 3, 1e4, 1152, 48, g_dtype=ms.MS_BF16)
    assert not torch.equal(a["A"], c["A"])


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (16, 1e3), (128, 1e5)])
def test_generator_conditioning_and_mixing(ms, n, kappa):
    d = 65536 if n < 128 else 32768
    print("gen conditioning d=%d n=%d kappa=%g" % (d, n, kappa), flush=True)
    t = ms.gen_lstsq_request(7 + n, d, n, 2, kappa, 2 * n * n, 2 * n)
    torch.cuda.synchronize()
    A = to_host(t["A"]).astype(np.float64)
    D = np.logspace(0.0, -np.log10(kappa), n) if n > 1 else np.ones(1)
    sv = np.linalg.svd(A / np.sqrt(d), compute_uv=False)
    eps = np.sqrt(n / d)
    ratio = sv / D                      # both descending
    assert np.all(ratio > 1 - 3 * eps - 1e-3) and np.all(ratio < 1 + 3 * eps + 1e-3), \
        (ratio.min(), ratio.max())
    if n > 1:
        M = A.T @ A
        off = M - np.diag(np.diag(M))
        assert np.linalg.norm(off) > 0.05 * np.linalg.norm(M)
    # Gaussian entries: the first column of Z diag(D) Q is a Gaussian column
    col = A[:, 0] / A[:, 0].std()
    skew = np.mean(col ** 3)
    kurt = np.mean(col ** 4)
    assert abs(skew) < 0.05 and abs(kurt - 3.0) < 0.1, (skew, kurt)


def test_generator_rhs_codes_and_gaussian(ms):
    d, n, nrhs, k, k2 = 200000, 16, 8, 4096, 32
    print("gen rhs/codes d=%d n=%d nrhs=%d" % (d, n, nrhs), flush=True)
    t = ms.gen_lstsq_request(5, d, n, nrhs, 1e2, k, k2, g_dtype=ms.MS_F32)
    tb = ms.gen_lstsq_request(5, d, n, nrhs, 1e2, k, k2, g_dtype=ms.MS_BF16, want=("G",))
    t64 = ms.gen_lstsq_request(5, d, n, nrhs, 1e2, k, k2, g_dtype=ms.MS_F64, want=("G",))
    torch.cuda.synchronize()
    A = to_host(t["A"]).astype(np.float64)
    B = to_host(t["B"]).astype(np.float64)
    xs = to_host(t["xstar"]).astype(np.float64)
    assert xs.shape == (n, nrhs)
    R = B - A @ xs
    rms = np.sqrt(np.mean(R ** 2))
    assert 0.8e-6 < rms < 3e-6 and np.abs(R).max() < 1e-4, rms
    xv = xs.ravel()
    assert abs(xv.mean()) < 0.4 and 0.6 < xv.std() < 1.4
    h = to_host(t["h"]).astype(np.int64)
    s = to_host(t["s"]).astype(np.int64)
    assert h.min() >= 0 and h.max() < k
    cnt = np.bincount(h, minlength=k)
    chi2 = np.sum((cnt - d / k) ** 2 / (d / k))
    assert chi2 < k + 6 * np.sqrt(2 * k), chi2     # k - 1 degrees of freedom
    assert set(np.unique(s)) == {-1, 1} and abs(s.mean()) < 5 / np.sqrt(d)
    G = t["G"]
    assert G.shape == (k2, k) and G.stride(0) == 1
    g = to_host(G).astype(np.float64).ravel()
    assert abs(g.mean()) < 5 / np.sqrt(g.size * k2)
    assert abs(g.var() * k2 - 1.0) < 0.02
    assert torch.equal(G.to(torch.bfloat16), tb["G"])
    assert torch.equal(G.to(torch.float64), t64["G"])
