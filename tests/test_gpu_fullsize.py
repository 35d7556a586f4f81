"""GPU parity at the full sizes of the FP32 workloads, in the configuration
the library runs by default:

* ill-conditioned FP32 least squares: A = Z diag(logspace(0, -6, 128)) Q,
  16,777,216 x 128, one right-hand side, k = 32,768, k2 = 256;
* mixed precision: A = Z diag(logspace(0, -4, 256)) FP32, 8,388,608 x 256,
  four right-hand sides, k = 131,072, BF16 Gaussian stage 512 x 131,072,
  FP64 QR, three FP64-residual refinement steps.

Checks: the CountSketch on sampled buckets (the oracle folds exactly those
buckets' rows: FP32 LDS mode within 1e-5 normwise, the deterministic sorted
mode bit for bit); the FP32 solution after one FP64-residual refinement step
by its residual ratio against the FP64 least-squares optimum (blocked
Householder QR of [A | b]), rho <= 2; the mixed-precision solution against the oracle's
FP64 sketch-and-solve with the same (h, s, G) within the bound the
refinement reaches at three steps (1e-5).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import bf16_dev, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


def _sampled_buckets(orc, A, h, s, k, buckets):
    """Oracle CountSketch rows of the given buckets (ascending-row fold in the
    data's precision), from only those buckets' rows."""
    sel = np.isin(h, buckets)
    idx = np.nonzero(sel)[0]                      # ascending rows
    remap = np.full(k, -1, dtype=np.int64)
    remap[buckets] = np.arange(len(buckets))
    hs = remap[h[idx]].astype(np.int32)
    return orc.countsketch(np.asfortranarray(A[idx]), hs, s[idx], len(buckets))


def _check_sampled_countsketch(ms, orc, A, Ad, h, hd, s, sd, k, seed):
    rng = np.random.default_rng(seed)
    buckets = np.sort(rng.choice(k, size=64, replace=False))
    Yo = _sampled_buckets(orc, A, h, s, k, buckets)
    for mode in ("lds", "sorted"):
        print("countsketch sampled, mode", mode, flush=True)
        Y, ws = ms.countsketch_apply(Ad, hd, sd, k, mode=mode)
        ms.check_status(ws)
        Ys = to_host(Y[torch.from_numpy(buckets).to(Y.device)])
        if mode == "sorted":
            assert np.array_equal(Ys.view(np.uint32), Yo.view(np.uint32)), mode
        else:
            assert rel(Ys, Yo) <= 1e-5, (mode, rel(Ys, Yo))
        del Y, ws
        torch.cuda.empty_cache()


def test_fp32_ill_conditioned_full_size(ms, orc):
    d, n, nrhs, k, k2, seed = 1 << 24, 128, 1, 32768, 256, 32
    print("generate A %d x %d (kappa 1e6)" % (d, n), flush=True)
    A = synth.conditioned_matrix(d, n, 1e6, seed=seed, dtype=np.float32)
    B, _ = synth.lstsq_rhs(A, nrhs, seed=seed)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype="f32")
    Ad, Bd, hd, sd, Gd = to_dev(A), to_dev(B), to_dev(h), to_dev(s), to_dev(G)
    _check_sampled_countsketch(ms, orc, A, Ad, h, hd, s, sd, k, seed)
    print("sketch_lstsq FP32 full size, first pass and one refinement step", flush=True)
    X0, ws = ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k)
    ms.check_status(ws)
    X0 = to_host(X0)
    X1, ws = ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k, refine_steps=1)
    ms.check_status(ws)
    X1 = to_host(X1)
    del Ad, Bd, ws
    torch.cuda.empty_cache()
    _, rt = orc.lstsq_tsqr(A, B)

    def resid(Xv):
        r = B.astype(np.float64).copy()
        for r0 in range(0, d, 1 << 20):
            r[r0:r0 + (1 << 20)] -= A[r0:r0 + (1 << 20)].astype(np.float64) @ Xv
        return np.linalg.norm(r)

    rho_0, rho_1 = resid(X0) / rt[0], resid(X1) / rt[0]
    print("rho first pass %.4f, one refinement step %.4f" % (rho_0, rho_1))
    # At kappa = 1e6 the FP32 sketch of b carries rounding of order u32 ||b||,
    # comparable with the sketched 1e-6 noise, so the first pass sits near
    # rho = 2 (reported, not asserted).  One FP64-residual refinement step
    # takes X to the FP64 sketch-and-solve fixed point up to a kappa * u32
    # perturbation of Q: the residual criterion rho <= 2 holds.
    assert 1.0 - 1e-6 <= rho_1 <= 2.0


def test_mixed_precision_full_size(ms, orc):
    d, n, nrhs, k, k2, seed = 1 << 23, 256, 4, 131072, 512, 33
    print("generate A %d x %d (column scales 1 .. 1e-4)" % (d, n), flush=True)
    A = synth.conditioned_matrix(d, n, 1e4, seed=seed, dtype=np.float32, rotate=False)
    B, _ = synth.lstsq_rhs(A, nrhs, seed=seed)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype="bf16")
    Ad, Bd, hd, sd = to_dev(A), to_dev(B), to_dev(h), to_dev(s)
    _check_sampled_countsketch(ms, orc, A, Ad, h, hd, s, sd, k, seed)
    print("sketch_lstsq mixed precision full size, 3 refinement steps", flush=True)
    X, ws = ms.sketch_lstsq(Ad, Bd, hd, sd, bf16_dev(G), k, refine_steps=3)
    ms.check_status(ws)
    X = to_host(X)
    del Ad, Bd, ws
    torch.cuda.empty_cache()
    print("oracle FP64 sketch-and-solve", flush=True)
    A64 = np.asfortranarray(A, dtype=np.float64)
    del A
    X64, _, _ = orc.sketch_lstsq(A64, B.astype(np.float64), h, s, G.astype(np.float64), k)
    err = rel(X, X64)
    print("mixed precision vs FP64 sketch-and-solve: %.3e" % err)
    assert np.isfinite(X).all() and err <= 1e-5
