"""GPU parity: Gaussian stage (MFMA), multisketch, Householder QR solve and
the composite sketch-and-solve, against the oracle through the C ABI.

Bar: normwise relative 1e-12 for FP64 results and 1e-5 for FP32 results
(the Gaussian stage in FP32, or BF16 products with FP32 accumulation against
the oracle's FP64 sum of the same BF16 operands).  The least-squares solution
of a well-conditioned FP64 problem is held to 1e-12; ill-conditioned FP32
problems are judged by their residual ratio, since their forward error is of
order kappa * u32 on both sides.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import bf16_dev, g_dev, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


# ------------------------------------------------------------------- Gaussian stage
GEMM_CASES = [
    # k2, k, ncols
    (16, 128, 9),
    (37, 1000, 13),     # ragged in every dimension
    (128, 8192, 65),    # the 128 x 8192 stage of the FP64 workload
    (64, 2048, 1),
    (256, 32768, 129),  # the 256 x 32768 stage of the FP32 workload
    (300, 4100, 150),   # two row tiles and two column tiles of the 16-bit kernel, ragged
    (257, 777, 145),    # second row tile of one row, second column tile of one column
]


@pytest.mark.parametrize("k2,k,nc", GEMM_CASES)
@pytest.mark.parametrize("gd", ["f64", "f32", "bf16", "f16"])
def test_gaussian_stage_parity(ms, orc, k2, k, nc, gd):
    print("gaussian %s k2=%d k=%d nc=%d" % (gd, k2, k, nc), flush=True)
    G = synth.gaussian_sketch(k2, k, seed=k2 + k, dtype=gd)
    ydt = np.float64 if gd == "f64" else np.float32
    Y = synth.normal_matrix(k, nc, seed=nc + 7, dtype=ydt)
    if gd == "f16":
        # columns of very different scales: the FP16 stage's per-column scale
        Y = np.asfortranarray(Y * np.logspace(-20, 20, nc, dtype=np.float64)[None, :]
                              .astype(np.float32))
    Z, ws = ms.gaussian_apply(g_dev(G, gd), to_dev(Y))
    ms.check_status(ws)
    Yref = {"bf16": orc.round_bf16, "f16": orc.round_f16_colscaled}.get(gd, lambda y: y)(Y)
    Zr = orc.gemm(G, Yref)
    assert rel(to_host(Z), Zr) <= (1e-12 if gd == "f64" else 1e-5)


def test_gaussian_stage_bf16_full_width_sampled(ms, orc):
    # the 512 x 131072 BF16 stage on 260 columns; the oracle checks 4 of them
    k2, k, nc = 512, 131072, 260
    G = synth.gaussian_sketch(k2, k, seed=3, dtype="bf16")
    Y = synth.normal_matrix(k, nc, seed=4, dtype=np.float32)
    Z, ws = ms.gaussian_apply(bf16_dev(G), to_dev(Y))
    ms.check_status(ws)
    cols = [0, 131, 258, 259]
    Zr = orc.gemm(G, orc.round_bf16(Y[:, cols]))
    assert rel(to_host(Z)[:, cols], Zr) <= 1e-5


def test_gaussian_identity_exact(ms):
    # G = I (k2 = k): Z = Y bit for bit in FP64
    k, nc = 64, 5
    Y = synth.normal_matrix(k, nc, seed=5)
    Z, ws = ms.gaussian_apply(to_dev(np.eye(k)), to_dev(Y))
    ms.check_status(ws)
    assert np.array_equal(to_host(Z), Y)


@pytest.mark.parametrize("mode", ["lds", "sorted"])
@pytest.mark.parametrize("d,n,k,k2,gd,yt", [(20000, 8, 128, 16, "f64", 0),
                                            (100003, 16, 512, 32, "f32", 0),
                                            (100003, 16, 512, 32, "bf16", 3),
                                            (100003, 16, 512, 32, "bf16", 1),
                                            (100003, 16, 512, 32, "f16", 3),
                                            (100003, 16, 512, 32, "f16", 1)])
def test_multisketch_parity(ms, orc, mode, d, n, k, k2, gd, yt):
    dt = np.float64 if gd == "f64" else np.float32
    A = synth.normal_matrix(d, n, seed=d, dtype=dt)
    h = synth.bucket_map(d, k, seed=d)
    s = synth.signs(d, seed=d)
    G = synth.gaussian_sketch(k2, k, seed=d, dtype=gd)
    Gd = g_dev(G, gd)
    Z, ws = ms.multisketch_apply(to_dev(A), to_dev(h), to_dev(s), Gd, k, mode=mode, y_terms=yt)
    ms.check_status(ws)
    Y = orc.countsketch(A, h, s, k)
    # BF16 G with three Y terms: the terms sum to the GPU's FP32 sketch
    # exactly, so Z is G Y itself (FP32 bar); with one term Y is rounded to
    # BF16, and with the LDS sketch the GPU's FP32 sketch differs from the
    # oracle's in its last bits (association order), so the few entries next
    # to a BF16 rounding boundary may round to the neighbouring BF16 value (a
    # 2^-8 relative change of those entries): 1e-3
    # (FP16: the same with FP16's 2^-11 rounding step instead of 2^-8: 1e-4)
    rnd = {"bf16": orc.round_bf16, "f16": orc.round_f16_colscaled}.get(gd)
    Zr = orc.gemm(G, rnd(Y) if (rnd is not None and yt == 1) else Y)
    exact = mode == "sorted" or yt == 3
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5 if exact else 1e-3,
           "f16": 1e-5 if exact else 1e-4}[gd]
    assert rel(to_host(Z), Zr) <= tol


# ------------------------------------------------------------------- QR solve
QR_CASES = [(1, 1, 1), (16, 8, 1), (37, 19, 3), (128, 64, 1), (64, 64, 2), (256, 128, 1),
            (512, 256, 4),
            # panelled (blocked) factorisation: ragged last panel, 3 row classes
            (300, 150, 2), (1000, 200, 3), (1024, 512, 1), (257, 33, 8),
            # single-workgroup paths: LDS-resident, and global memory beyond 1024 rows
            (700, 17, 1), (1100, 40, 2)]


@pytest.mark.parametrize("m,n,nrhs", QR_CASES)
def test_qr_solve_parity(ms, orc, m, n, nrhs):
    print("qr m=%d n=%d nrhs=%d" % (m, n, nrhs), flush=True)
    W = synth.normal_matrix(m, n, seed=m + n)
    B = synth.normal_matrix(m, nrhs, seed=m + n + 1)
    X, R, ws = ms.qr_solve(to_dev(W), to_dev(B), want_r=True)
    ms.check_status(ws)
    Xr = orc.qr_solve(W, B)
    F, _ = orc.householder_qr(W)
    Rr = np.triu(F[:n, :n])
    kappa = np.linalg.cond(W)
    assert rel(to_host(X), Xr) <= max(1e-12, 10 * kappa * 1e-16 * n)
    assert rel(to_host(R), Rr) <= 1e-13 * n


@pytest.mark.parametrize("m,n,zero", [(20, 4, 2), (600, 200, 37)])
def test_qr_solve_singular(ms, m, n, zero):
    W = synth.normal_matrix(m, n, seed=7)
    W[:, zero] = 0.0
    X, _, ws = ms.qr_solve(to_dev(W), to_dev(np.ones((m, 1))))
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_SINGULAR
    assert np.isnan(to_host(X)).all()


# ------------------------------------------------------------------- sketch-and-solve
def _lstsq_inputs(d, n, nrhs, k, k2, seed, dtype=np.float64, gd="f64", kappa=None, noise=1e-6):
    if kappa is None:
        A = synth.normal_matrix(d, n, seed=seed, dtype=dtype)
    else:
        A = synth.conditioned_matrix(d, n, kappa, seed=seed, dtype=dtype)
    B, xs = synth.lstsq_rhs(A, nrhs, seed=seed, noise=noise)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype=gd)
    return A, B, xs, h, s, G


def _gpu_lstsq(ms, A, B, h, s, G, k, gd="f64", **kw):
    Gd = g_dev(G, gd)
    X, ws = ms.sketch_lstsq(to_dev(A), to_dev(B), to_dev(h), to_dev(s), Gd, k, **kw)
    ms.check_status(ws)
    return to_host(X)


@pytest.mark.parametrize("mode", ["lds", "sorted", "atomic"])
@pytest.mark.parametrize("d,n,nrhs", [(4096, 4, 1), (50001, 8, 3), (200000, 16, 8)])
def test_lstsq_fp64_parity(ms, orc, mode, d, n, nrhs):
    k, k2 = 2 * n * n, 2 * n
    A, B, xs, h, s, G = _lstsq_inputs(d, n, nrhs, k, k2, seed=d + n)
    X = _gpu_lstsq(ms, A, B, h, s, G, k, mode=mode)
    Xr, _, _ = orc.sketch_lstsq(A, B, h, s, G, k)
    assert rel(X, Xr) <= 1e-12


def test_lstsq_fp64_full_workload(ms, orc):
    # A 4,194,304 x 64 FP64, b = A x* + 1e-6 N(0,1), k = 8192, G 128 x 8192
    d, n, nrhs, k, k2 = 4194304, 64, 1, 8192, 128
    print("lstsq full d=%d n=%d" % (d, n), flush=True)
    A, B, xs, h, s, G = _lstsq_inputs(d, n, nrhs, k, k2, seed=14209)
    X = _gpu_lstsq(ms, A, B, h, s, G, k)
    Xr, _, _ = orc.sketch_lstsq(A, B, h, s, G, k)
    assert rel(X, Xr) <= 1e-12
    # residual ratio against the full least-squares optimum (LAPACK)
    xt = np.linalg.lstsq(A, B, rcond=None)[0]
    rho = np.linalg.norm(B - A @ X) / np.linalg.norm(B - A @ xt)
    print("rho =", rho)
    assert 1.0 - 1e-9 <= rho <= 2.0


@pytest.mark.parametrize("d,n,nrhs,k", [(3000, 16, 2, 512), (100, 8, 1, 128), (5000, 8, 1, 128)])
def test_lstsq_edge_shapes(ms, orc, d, n, nrhs, k):
    # k > d (sketch does not shrink rows) and a square Gaussian stage (k2 = n)
    k2 = n if d == 5000 else 2 * n
    A, B, xs, h, s, G = _lstsq_inputs(d, n, nrhs, k, k2, seed=d + 1)
    X = _gpu_lstsq(ms, A, B, h, s, G, k)
    Xr, _, Zr = orc.sketch_lstsq(A, B, h, s, G, k)
    # a square Gaussian stage (k2 = n) gives an ill-conditioned sketch: both
    # sides solve the same FP64 system up to association order, so X agrees
    # to about kappa(Z_A) * u64 (times a small factor for the QR and the
    # sums), never looser than the FP64 bar of 1e-12 for kappa(Z_A) <= 100
    kz = np.linalg.cond(Zr[:, :n])
    tol = max(1e-12, 100 * kz * 2.0 ** -53)
    print("edge d=%d n=%d k=%d k2=%d: kappa(Z_A) %.3g, err %.3e, tol %.3e"
          % (d, n, k, k2, kz, rel(X, Xr), tol))
    assert rel(X, Xr) <= tol


def test_lstsq_consistent_exact_recovery(ms):
    d, n, k, k2 = 100000, 16, 512, 32
    A, B, xs, h, s, G = _lstsq_inputs(d, n, 2, k, k2, seed=3, noise=0.0)
    X = _gpu_lstsq(ms, A, B, h, s, G, k)
    assert rel(X, xs) <= 1e-12


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_lstsq_fp32_well_conditioned(ms, orc, seed):
    # kappa(A) ~ 1, FP32 data and FP32 Gaussian stage.  The reference sketch
    # is Def. 3's exact sum rounded once to FP32 (the GPU's LDS variant sums
    # each workgroup's rows in FP64 and rounds its partial once), so the two
    # sketches differ by a few FP32 roundings (~1e-7 relative) and X by
    # kappa(Z_A) (~6 for k2 = 2n) times that: the FP32 bar of 1e-5 binds.
    d, n, nrhs, k, k2 = 1 << 20, 32, 1, 2048, 64
    A, B, xs, h, s, G = _lstsq_inputs(d, n, nrhs, k, k2, seed=seed, dtype=np.float32, gd="f32")
    X = _gpu_lstsq(ms, A, B, h, s, G, k, gd="f32")
    Xr, _, _ = orc.sketch_lstsq(A, B, h, s, G, k, y_acc64=True)
    Xf, _, _ = orc.sketch_lstsq(A, B, h, s, G, k)
    print("fp32 kappa~1 seed %d: err vs exact-sum sketch %.3e, vs FP32-fold sketch %.3e"
          % (seed, rel(X, Xr), rel(X, Xf)))
    assert rel(X, Xr) <= 1e-5


def test_lstsq_fp32_ill_conditioned_residual(ms, orc):
    # A = Z D Q with kappa 1e6, FP32, b = A x* + 1e-6 N(0,1).  The FP32
    # sketch of b carries rounding of order u32 ||b||, comparable with the
    # sketched noise, so the first-pass solution's residual ratio depends on
    # those roundings (it sits near 2).  One FP64-residual refinement step
    # removes them: its fixed point satisfies Q^T G C (b - A x) = 0 with the
    # FP64 residual, i.e. the FP64 sketch-and-solve solution of the stored
    # data up to the perturbation of Q by the FP32 sketch (a relative change
    # of the residual of order kappa * u32 = 0.06).  Bars: rho <= 2 (the
    # residual criterion) and within 10% of the FP64 sketch-and-solve rho.
    d, n, nrhs, k, k2 = 1 << 20, 32, 1, 2048, 64
    A, B, xs, h, s, G = _lstsq_inputs(d, n, nrhs, k, k2, seed=12, dtype=np.float32, gd="f32",
                                      kappa=1e6)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    xt = np.linalg.lstsq(A64, B64, rcond=None)[0]
    rt = np.linalg.norm(B64 - A64 @ xt)
    X64, _, _ = orc.sketch_lstsq(A64, B64, h, s, G.astype(np.float64), k)
    rho_64 = np.linalg.norm(B64 - A64 @ X64) / rt
    X0 = _gpu_lstsq(ms, A, B, h, s, G, k, gd="f32")
    X1 = _gpu_lstsq(ms, A, B, h, s, G, k, gd="f32", refine_steps=1)
    rho_0 = np.linalg.norm(B64 - A64 @ X0) / rt
    rho_1 = np.linalg.norm(B64 - A64 @ X1) / rt
    print("rho: first pass %.4f, one refinement step %.4f, FP64 sketch-and-solve %.4f"
          % (rho_0, rho_1, rho_64))
    assert 1.0 - 1e-6 <= rho_1 <= 2.0
    assert abs(rho_1 - rho_64) <= 0.1 * rho_64


@pytest.mark.parametrize("yt", [1, 3])
@pytest.mark.parametrize("refine", [0, 1, 2, 3])
def test_lstsq_bf16_refinement(ms, orc, refine, yt):
    # FP32 A with column scales down to 1e-4, BF16 Gaussian stage, FP64 QR,
    # FP64-residual refinement steps.  Without refinement the BF16 rounding of
    # the sketched right-hand side costs about u_bf16 * (column scale ratio)
    # in the small-scale components of x (relative error O(1)); each step
    # contracts the error by about u_bf16 * kappa(column-scaled sketch)
    # (~1e-3); the fixed point differs from the FP64 sketch-and-solve solution
    # by a term proportional to the sketched residual (~1e-6 here, set by the
    # 1e-6 noise of b).  The same iteration on the CPU oracle gives
    # 1.31, 3.6e-3, 4.2e-6, 1.24e-6 for 0..3 steps on this problem.
    d, n, nrhs, k, k2 = 1 << 19, 32, 4, 2048, 64
    seed = 21
    Z = synth.normal_matrix(d, n, seed=seed, dtype=np.float64)
    A = np.asfortranarray((Z * np.logspace(0, -4, n)[None, :]).astype(np.float32))
    B, xs = synth.lstsq_rhs(A, nrhs, seed=seed)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype="bf16")
    X = _gpu_lstsq(ms, A, B, h, s, G, k, gd="bf16", refine_steps=refine, y_terms=yt)
    # the FP64 sketch-and-solve solution with the same (h, s, G)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    X64, _, _ = orc.sketch_lstsq(A64, B64, h, s, G.astype(np.float64), k)
    err = rel(X, X64)
    xt = np.linalg.lstsq(A64, B64, rcond=None)[0]
    rho = np.linalg.norm(B64 - A64 @ X) / np.linalg.norm(B64 - A64 @ xt)
    print("y_terms=%d refine=%d err vs FP64 sketch-and-solve = %.3e, rho = %.4f"
          % (yt, refine, err, rho))
    # three exact BF16 terms: the first pass carries only the FP32 sketch's
    # rounding (kappa * u32 ~ 1e-3 in the small-scale components), which each
    # step contracts by ~kappa * u32 as well
    bound = ({0: 5.0, 1: 1e-2, 2: 1e-4, 3: 1e-5} if yt == 1 else
             {0: 1e-2, 1: 1e-5, 2: 1e-5, 3: 1e-5})[refine]
    assert np.isfinite(X).all() and err <= bound
    if refine >= 2:
        assert rho <= 2.0


@pytest.mark.parametrize("yt", [1, 3])
@pytest.mark.parametrize("refine", [0, 1, 2])
def test_lstsq_f16_refinement(ms, orc, refine, yt):
    # the problem of test_lstsq_bf16_refinement with an FP16 Gaussian stage
    # (per-column power-of-two scale, then FP16).  The same iteration on the
    # CPU oracle (one FP16 term) gives 0.23, 6.2e-5, 2.3e-7 for 0..2 steps
    # (BF16: 1.31, 3.6e-3, 4.2e-6): FP16's 2^-11 rounding step against
    # BF16's 2^-8.  Bars: about 4x (first pass) and 16x those values; with
    # three exact terms the bars of the BF16 three-term case.
    d, n, nrhs, k, k2 = 1 << 19, 32, 4, 2048, 64
    seed = 21
    Z = synth.normal_matrix(d, n, seed=seed, dtype=np.float64)
    A = np.asfortranarray((Z * np.logspace(0, -4, n)[None, :]).astype(np.float32))
    B, xs = synth.lstsq_rhs(A, nrhs, seed=seed)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype="f16")
    X = _gpu_lstsq(ms, A, B, h, s, G, k, gd="f16", refine_steps=refine, y_terms=yt)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    X64, _, _ = orc.sketch_lstsq(A64, B64, h, s, G.astype(np.float64), k)
    err = rel(X, X64)
    print("f16 y_terms=%d refine=%d err vs FP64 sketch-and-solve = %.3e" % (yt, refine, err))
    bound = ({0: 1.0, 1: 1e-3, 2: 4e-6} if yt == 1 else {0: 1e-2, 1: 1e-5, 2: 1e-5})[refine]
    assert np.isfinite(X).all() and err <= bound


def test_lstsq_range_error(ms):
    d, n, k, k2 = 1000, 4, 32, 8
    A, B, xs, h, s, G = _lstsq_inputs(d, n, 1, k, k2, seed=2)
    h[10] = -1
    Gd = to_dev(G)
    X, ws = ms.sketch_lstsq(to_dev(A), to_dev(B), to_dev(h), to_dev(s), Gd, k)
    with pytest.raises(ms.MsketchError) as e:
        ms.check_status(ws)
    assert e.value.code == ms.MS_ERR_RANGE


@pytest.mark.parametrize("d,n,nrhs,k2", [(5000, 8, 1, 64), (30000, 13, 3, 96),
                                         (30000, 40, 8, 200), (40000, 64, 2, 512),
                                         (20000, 20, 1, 520)])
def test_lstsq_fp64_refinement_fixed_point(ms, orc, d, n, nrhs, k2):
    # FP64 data and G: the first pass is the FP64 sketch-and-solve solution,
    # whose sketched residual S r is orthogonal to range(S A), so each
    # refinement step's correction R^{-1} (Q^T S r)[0:n) is zero up to
    # rounding and X stays the oracle's solution.  A wrong reflector
    # application or back substitution in the refinement step moves X by
    # about ||S r|| / ||R|| (the 1e-6 noise of b): far outside the bar.
    # Shapes: every register width of the staged refinement kernel (k2 up to
    # 64, 128, 256, 512), blocks of eight reflectors with a ragged last one,
    # one to eight right-hand sides, and k2 > 512 (the unstaged kernel).
    k = 4096
    print("fp64 refinement d=%d n=%d nrhs=%d k2=%d" % (d, n, nrhs, k2), flush=True)
    A, B, xs, h, s, G = _lstsq_inputs(d, n, nrhs, k, k2, seed=d + k2)
    X = _gpu_lstsq(ms, A, B, h, s, G, k, refine_steps=2)
    Xr, _, _ = orc.sketch_lstsq(A, B, h, s, G, k)
    assert rel(X, Xr) <= 1e-10
