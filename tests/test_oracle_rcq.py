"""Pins of the rand_cholQR least-squares oracle (Alg. 5, Sec. 6.3, with the
multisketch S = G C as the sketch operator).

What the mathematics fixes, independent of the oracle's own code:
* the result is the least-squares optimum of min ||B - A X|| (no sketch
  distortion), so it matches LAPACK's least-squares solver within the
  backward-stable error bound, whatever the sketch;
* R is an R factor of A: R^T R = A^T A, R upper triangular, Q = A R^{-1} has
  orthonormal columns;
* with the sketch replaced by A itself (S = I), R0 is already an R factor of
  A, Q0 is orthonormal and the Cholesky factor R1 is the identity, so R = R0;
* two different sketches give the same X, while sketch-and-solve (Alg. 1)
  moves with the sketch.
"""
import numpy as np
import pytest

import synth

pytestmark = []


def _problem(d, n, nrhs, kappa, seed, noise=1e-3):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((d, n))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Z @ np.diag(np.logspace(0, -np.log10(kappa), n)) @ Q
    x = rng.standard_normal((n, nrhs))
    B = A @ x + noise * rng.standard_normal((d, nrhs))
    return np.asfortranarray(A), np.asfortranarray(B)


def _sketch(d, n, seed):
    k, k2 = 2 * n * n, 2 * n
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype="f64")
    return h, s, G, k


@pytest.mark.parametrize("d,n,nrhs,kappa", [(2000, 4, 1, 1.0), (5000, 8, 3, 1e2),
                                            (8000, 16, 2, 1e4), (20000, 32, 1, 1e2)])
def test_rand_cholqr_is_the_least_squares_optimum(orc, d, n, nrhs, kappa):
    A, B = _problem(d, n, nrhs, kappa, seed=d + n)
    h, s, G, k = _sketch(d, n, seed=7 + n)
    X, R, _ = orc.rand_cholqr_lstsq(A, B, h, s, G, k)
    Xl = np.linalg.lstsq(A, B, rcond=None)[0]
    # backward-stable LS: error ~ u (kappa + kappa^2 ||r|| / (||A|| ||x||))
    tol = 1e-13 * kappa + 1e-14 * kappa * kappa * 1e-3
    assert np.linalg.norm(X - Xl) / np.linalg.norm(Xl) <= max(tol, 5e-14)


@pytest.mark.parametrize("d,n,kappa", [(3000, 8, 1.0), (6000, 16, 1e2)])
def test_rand_cholqr_R_factors_A(orc, d, n, kappa):
    A, B = _problem(d, n, 1, kappa, seed=11 + n)
    h, s, G, k = _sketch(d, n, seed=3)
    _, R, _ = orc.rand_cholqr_lstsq(A, B, h, s, G, k)
    assert np.all(np.tril(R, -1) == 0.0)
    AtA = A.T @ A
    assert np.linalg.norm(R.T @ R - AtA) / np.linalg.norm(AtA) <= 1e-13
    Q = np.linalg.solve(R.T, A.T).T               # Q = A R^{-1}
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-12 * kappa


def test_rand_cholqr_with_the_identity_sketch(orc):
    # S = I: R0 = the Householder R of A, Q0 = A R0^{-1} orthonormal, R1 = I
    A, B = _problem(400, 6, 2, 10.0, seed=5)
    X, R = orc.rand_cholqr_from_sketch(A, A, B)
    F, _ = orc.householder_qr(A)
    R0 = np.triu(F[:6, :6])
    assert np.linalg.norm(R - R0) / np.linalg.norm(R0) <= 1e-14
    Xl = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.linalg.norm(X - Xl) / np.linalg.norm(Xl) <= 1e-13


def test_rand_cholqr_does_not_depend_on_the_sketch(orc):
    d, n = 6000, 8
    A, B = _problem(d, n, 2, 1e2, seed=21, noise=1e-1)
    out, sas = [], []
    for seed in (1, 2):
        h, s, G, k = _sketch(d, n, seed=seed)
        out.append(orc.rand_cholqr_lstsq(A, B, h, s, G, k)[0])
        sas.append(orc.sketch_lstsq(A, B, h, s, G, k)[0])
    assert np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[0]) <= 1e-12
    # sketch-and-solve moves with the sketch (its O(1) distortion)
    assert np.linalg.norm(sas[0] - sas[1]) / np.linalg.norm(sas[0]) > 1e-6


def test_rand_cholqr_fp32_data_is_solved_in_fp64(orc):
    # FP32 A and B: the sketch in FP32 (here also rounded to BF16) only
    # preconditions; the result is the FP64 optimum of the stored values
    A, B = _problem(4000, 8, 2, 1e2, seed=31)
    A32, B32 = np.asfortranarray(A, dtype=np.float32), np.asfortranarray(B, dtype=np.float32)
    h, s, G, k = _sketch(4000, 8, seed=4)
    G32 = np.asarray(G, dtype=np.float32).astype(np.float64)
    X, _, _ = orc.rand_cholqr_lstsq(A32, B32, h, s, G32, k, y_bf16=True)
    Xl = np.linalg.lstsq(A32.astype(np.float64), B32.astype(np.float64), rcond=None)[0]
    assert np.linalg.norm(X - Xl) / np.linalg.norm(Xl) <= 1e-11
