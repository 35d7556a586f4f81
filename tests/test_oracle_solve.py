"""Pins for the oracle's Gaussian stage, Householder QR, solve, normal
equations and the composite multisketch sketch-and-solve (Alg. 1).

Pinned against: library matmul within Higham's dot-product bound, the identity
matrix, LAPACK's QR/least-squares, orthogonality and reconstruction, exact
recovery on consistent systems, the identity sketch, scale equivariance, the
residual-ratio lower bound and its Gaussian-sketch mean, and the paper's
conditioning experiment (normal equations break down where QR-based solvers
do not, Sec. 6.3).
"""
import numpy as np
import pytest

import synth

U64 = np.finfo(np.float64).eps / 2


# ---------------------------------------------------------------- Gaussian stage
def test_gemm_identity_exact(orc):
    Y = synth.normal_matrix(64, 7, seed=1)
    assert np.array_equal(orc.gemm(np.eye(64), Y), Y)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (5, 3, 11), (16, 9, 300), (40, 65, 512)])
def test_gemm_vs_matmul_within_higham_bound(orc, M, N, K):
    G = synth.normal_matrix(M, K, seed=M + K, stream="G")
    Y = synth.normal_matrix(K, N, seed=N + K)
    Z = orc.gemm(G, Y)
    ref = G @ Y
    gamma = K * U64 / (1 - K * U64)
    bound = 2 * gamma * (np.abs(G) @ np.abs(Y))
    assert Z.shape == (M, N)
    assert np.all(np.abs(Z - ref) <= bound)


def test_gemm_integer_exact(orc):
    g = np.random.default_rng(2)
    G = g.integers(-50, 50, (6, 40)).astype(np.float64)
    Y = g.integers(-50, 50, (40, 3)).astype(np.float64)
    assert np.array_equal(orc.gemm(G, Y), G @ Y)


def test_gaussian_stage_preserves_norm_in_expectation(orc):
    # G ~ N(0, 1/k2) entrywise (Sec. 1): E||G y||^2 = ||y||^2, Var = 2||y||^4/k2
    k, k2, T = 200, 16, 600
    y = synth.normal_matrix(k, 1, seed=3)
    ny2 = float((y[:, 0] ** 2).sum())
    vals = [float((orc.gemm(synth.gaussian_sketch(k2, k, seed=500 + t), y)[:, 0] ** 2).sum())
            for t in range(T)]
    assert abs(np.mean(vals) - ny2) <= 4 * np.sqrt(2 * ny2 ** 2 / k2 / T)


# ---------------------------------------------------------------- QR and solve
def explicit_q(orc, F, tau):
    m, n = F.shape
    return orc.apply_qt(F, tau, np.eye(m)).T[:, :n]


@pytest.mark.parametrize("m,n", [(1, 1), (5, 5), (16, 8), (128, 64), (300, 17)])
def test_householder_qr_orthogonal_and_reconstructs(orc, m, n):
    W = synth.normal_matrix(m, n, seed=m * n)
    F, tau = orc.householder_qr(W)
    R = np.triu(F[:n, :n])
    Q = explicit_q(orc, F, tau)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 20 * n * U64 * np.sqrt(n)
    assert np.linalg.norm(Q @ R - W) <= 20 * m * U64 * np.linalg.norm(W)
    # R is unique up to the signs of its rows: compare with LAPACK's
    Rl = np.linalg.qr(W, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rl), rtol=1e-10, atol=1e-12 * np.abs(Rl).max())
    # LAPACK geqr2 convention: tau = 0 when the tail below the diagonal is
    # empty or zero, otherwise tau = 1 - alpha/beta lies in [1, 2]
    nz = tau != 0
    assert np.all(tau[nz] >= 1.0 - 1e-15) and np.all(tau[nz] <= 2.0)
    if m == n:
        assert tau[-1] == 0.0


def test_qr_zero_tail_gives_identity_reflector(orc):
    W = np.triu(synth.normal_matrix(6, 4, seed=4))
    F, tau = orc.householder_qr(W)
    assert np.array_equal(tau, np.zeros(4))
    assert np.array_equal(np.triu(F[:4]), W[:4])


def test_trsv_upper_solves(orc):
    n = 30
    R = np.triu(synth.normal_matrix(n, n, seed=5)) + 5 * np.eye(n)
    B = synth.normal_matrix(n, 3, seed=6)
    X = orc.trsv_upper(R, B)
    assert np.linalg.norm(R @ X - B) <= 100 * n * U64 * np.linalg.norm(R) * np.linalg.norm(X)


def test_singular_r_reports_and_fills_nan(orc):
    W = synth.normal_matrix(20, 4, seed=7)
    W[:, 2] = 0.0
    with pytest.raises(orc.OracleError) as e:
        orc.qr_solve(W, np.ones((20, 1)))
    assert e.value.code == orc.ERR_SINGULAR


@pytest.mark.parametrize("kappa", [1.0, 1e3, 1e8])
def test_qr_solve_matches_lapack_lstsq(orc, kappa):
    d, n = 500, 12
    A = synth.conditioned_matrix(d, n, kappa, seed=8)
    B, _ = synth.lstsq_rhs(A, 2, seed=8, noise=1e-3)
    X = orc.qr_solve(A, B)
    Xl = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.linalg.norm(X - Xl) <= 50 * kappa * kappa * U64 * np.linalg.norm(Xl) + 1e3 * kappa * U64 * np.linalg.norm(Xl)
    # residual is optimal to working accuracy
    r = np.linalg.norm(B - A @ X)
    rl = np.linalg.norm(B - A @ Xl)
    assert r <= rl * (1 + 1e-10)


def test_normal_equations_well_conditioned(orc):
    d, n = 2000, 10
    A = synth.conditioned_matrix(d, n, 1e2, seed=9)
    B, _ = synth.lstsq_rhs(A, 3, seed=9, noise=1e-2)
    X = orc.normal_equations(A, B)
    Xl = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.linalg.norm(X - Xl) <= 1e-10 * np.linalg.norm(Xl)


# ---------------------------------------------------------------- composite
def _problem(d, n, nrhs, seed, kappa=1.0, noise=1e-6, dtype=np.float64):
    k, k2 = 2 * n * n, 2 * n
    A = synth.conditioned_matrix(d, n, kappa, seed=seed, dtype=dtype, rotate=kappa != 1.0) \
        if kappa != 1.0 else synth.normal_matrix(d, n, seed=seed, dtype=dtype)
    B, xs = synth.lstsq_rhs(A, nrhs, seed=seed, noise=noise)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed)
    return A, B, xs, h, s, G, k


@pytest.mark.parametrize("d,n,nrhs", [(4096, 4, 1), (20000, 8, 3), (30000, 16, 2)])
def test_exact_recovery_consistent_system(orc, d, n, nrhs):
    A, B, xs, h, s, G, k = _problem(d, n, nrhs, seed=d + n, noise=0.0)
    X, Y, Z = orc.sketch_lstsq(A, B, h, s, G, k)
    assert np.linalg.norm(X - xs) <= 1e-12 * np.linalg.norm(xs)
    assert Y.shape == (k, n + nrhs) and Z.shape == (2 * n, n + nrhs)


def test_identity_sketch_reduces_to_plain_qr(orc):
    d, n = 64, 5
    A = synth.normal_matrix(d, n, seed=10)
    B, _ = synth.lstsq_rhs(A, 2, seed=10, noise=0.1)
    X, Y, Z = orc.sketch_lstsq(A, B, np.arange(d, dtype=np.int32), np.ones(d, np.int8),
                               np.eye(d), d)
    assert np.array_equal(Y, np.hstack([A, B]))
    assert np.array_equal(Z, np.hstack([A, B]))
    assert np.array_equal(X, orc.qr_solve(A, B))
    Xl = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.linalg.norm(X - Xl) <= 1e-13 * np.linalg.norm(Xl)


def test_scale_equivariance_exact(orc):
    A, B, xs, h, s, G, k = _problem(8192, 8, 2, seed=11, noise=1e-2)
    X, _, _ = orc.sketch_lstsq(A, B, h, s, G, k)
    X2, _, _ = orc.sketch_lstsq(8.0 * A, 0.25 * B, h, s, G, k)
    assert np.array_equal(X2, X * (0.25 / 8.0))


def test_residual_ratio_at_least_one_and_mean(orc):
    # rho = ||b - A x_s|| / ||b - A x_t|| >= 1 always (x_t optimal).  For a
    # Gaussian sketch E[rho^2 - 1] = n / (k2 - n - 1); with k2 = 2n and the
    # CountSketch in front the multisketch stays close to it.
    n, d, T = 8, 4096, 300
    vals = []
    for t in range(T):
        A, B, _, h, s, G, k = _problem(d, n, 1, seed=2000 + t, noise=1.0)
        X, _, _ = orc.sketch_lstsq(A, B, h, s, G, k)
        xt = np.linalg.lstsq(A, B, rcond=None)[0]
        rho2 = (np.linalg.norm(B - A @ X) / np.linalg.norm(B - A @ xt)) ** 2
        assert rho2 >= 1.0 - 1e-12
        vals.append(rho2 - 1.0)
    expect = n / (2 * n - n - 1)
    assert abs(np.mean(vals) - expect) <= 0.25 * expect


def test_conditioning_experiment(orc):
    # Sec. 6.3: with b = A e, the normal equations lose accuracy as kappa(A)
    # grows past u^{-1/2} while sketch-and-solve behaves like QR.
    d, n = 1 << 14, 16
    k, k2 = 2 * n * n, 2 * n
    h = synth.bucket_map(d, k, seed=12)
    s = synth.signs(d, seed=12)
    G = synth.gaussian_sketch(k2, k, seed=12)
    for kappa in (1e2, 1e10):
        A = synth.conditioned_matrix(d, n, kappa, seed=12)
        b = synth.paper_rhs(A, seed=12)
        rel = lambda x: np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        xq = orc.qr_solve(A, b)
        xs, _, _ = orc.sketch_lstsq(A, b, h, s, G, k)
        try:
            rn = rel(orc.normal_equations(A, b))
        except orc.OracleError as e:
            assert e.code == orc.ERR_SINGULAR
            rn = np.inf
        assert rel(xq) < 1e-12 and rel(xs) < 1e-10
        if kappa == 1e2:
            assert rn < 1e-12
        else:
            assert rn > 1e3 * max(rel(xq), rel(xs))


def test_fp32_path_consistent_system(orc):
    d, n, nrhs = 16384, 8, 2
    A, B, xs, h, s, _, k = _problem(d, n, nrhs, seed=13, noise=0.0, dtype=np.float32)
    G = synth.gaussian_sketch(2 * n, k, seed=13, dtype="f32")
    X, Y, Z = orc.sketch_lstsq(A, B, h, s, G, k)
    assert Y.dtype == np.float32
    # FP32 rounding of B = A x* and of the sketch: forward error ~ u32 * kappa
    assert np.linalg.norm(X - xs) <= 1e-4 * np.linalg.norm(xs)
    Xb, Yb, _ = orc.sketch_lstsq(A, B, h, s, synth.gaussian_sketch(2 * n, k, seed=13, dtype="bf16"),
                                 k, y_bf16=True)
    assert np.linalg.norm(Xb - xs) <= 5e-2 * np.linalg.norm(xs)
    assert np.array_equal(Yb, Y)  # the FP32 sketch itself is unrounded


def test_round_bf16_definition(orc):
    # RNE to 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8
    # is a tie -> even (1 + 2^-6); 1 + 2^-8 + 2^-20 rounds up.
    cases = {1.0: 1.0, 1.0 + 2 ** -8: 1.0, 1.0 + 3 * 2 ** -8: 1.0 + 2 ** -6,
             1.0 + 2 ** -8 + 2 ** -20: 1.0 + 2 ** -7, -3.0: -3.0,
             65504.0: 65536.0}
    for x, want in cases.items():
        got = float(orc.round_bf16(np.float32(x)))
        assert got == want, (x, got, want)
    x = synth.normal_matrix(1000, 1, seed=14, dtype=np.float32)[:, 0]
    assert np.array_equal(orc.round_bf16(x), synth.to_bf16_values(x))
    assert np.all(np.abs(orc.round_bf16(x) - x) <= np.abs(x) * 2.0 ** -8)


def test_lstsq_tsqr_matches_lapack_and_exact_cases(orc):
    # the blocked QR optimum equals LAPACK's least squares (SVD driver) on a
    # problem split over several row blocks, including a ragged last block
    rng = np.random.default_rng(5)
    d, n, nrhs = 1000, 7, 3
    A = rng.standard_normal((d, n)) * np.logspace(0, -3, n)
    B = rng.standard_normal((d, nrhs))
    X, res = orc.lstsq_tsqr(A, B, block_rows=96)
    Xl, _, _, _ = np.linalg.lstsq(A, B, rcond=None)
    assert np.allclose(X, Xl, rtol=1e-10, atol=1e-12)
    assert np.allclose(res, np.linalg.norm(B - A @ Xl, axis=0), rtol=1e-10)
    # consistent system: zero residual, exact solution
    xs = rng.standard_normal((n, 1))
    X2, res2 = orc.lstsq_tsqr(A, A @ xs, block_rows=128)
    assert np.allclose(X2, xs, rtol=1e-9) and res2[0] <= 1e-10 * np.linalg.norm(A @ xs)
    # b orthogonal to range(A): x = 0 and the residual is ||b||
    q, _ = np.linalg.qr(np.hstack([A, rng.standard_normal((d, 1))]))
    b = q[:, -1:]
    X3, res3 = orc.lstsq_tsqr(A, b, block_rows=300)
    assert np.abs(X3).max() <= 1e-10 and abs(res3[0] - 1.0) <= 1e-12


def test_fp32_path_acc64_sketch_is_correctly_rounded_exact_sum(orc):
    # With y_acc64 the FP32 sketch is Def. 3's exact bucket sum rounded once
    # to FP32: math.fsum gives the correctly rounded FP64 value of each exact
    # sum (A's and B's columns alike), which then rounds to the same FP32.
    import math
    d, n, nrhs, k, k2 = 3000, 3, 2, 48, 8
    A = synth.normal_matrix(d, n, seed=31, dtype=np.float32)
    B = synth.normal_matrix(d, nrhs, seed=32, dtype=np.float32)
    h = synth.bucket_map(d, k, seed=31)
    s = synth.signs(d, seed=31)
    G = synth.gaussian_sketch(k2, k, seed=31)
    X, Y, Z = orc.sketch_lstsq(A, B, h, s, G, k, y_acc64=True)
    AB = np.hstack([A, B]).astype(np.float64)
    expect = np.zeros((k, n + nrhs), np.float32)
    for m in range(k):
        rows = np.nonzero(h == m)[0]
        for c in range(n + nrhs):
            expect[m, c] = np.float32(math.fsum(float(s[i]) * AB[i, c] for i in rows))
    assert np.array_equal(Y, expect)
    # the rest of the path takes those values: Z = G Y in FP64
    assert np.allclose(Z, G @ Y.astype(np.float64), rtol=0, atol=1e-12 * np.abs(Z).max())
    # the FP32 fold of the same data is a different (less accurate) sketch
    _, Y32, _ = orc.sketch_lstsq(A, B, h, s, G, k)
    assert not np.array_equal(Y32, Y)
    assert np.abs(Y32.astype(np.float64) - expect).max() < 1e-5 * np.abs(expect).max()
