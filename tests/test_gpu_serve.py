"""GPU checks of the continuous-batching serving loop: every request of a
stream is solved, batches overlap with arrivals, each result is the same
alone and in the mix, and sampled requests match the oracle.

Alone vs in the mix: the batched call and a single sketch_lstsq differ only
in association order (LDS/atomic order of the FP32 sketch, K split of the
Gaussian stage), so X may move by about kappa * u32 between them, and the
residual b - A X by about kappa * u32 * ||b||.  The stated FP32 tolerance
1e-5 is therefore applied scaled by the request's condition number:
||X_mix - X_alone|| <= 1e-5 * kappa * ||X_alone|| and
| ||r_mix|| - ||r_alone|| | <= 1e-5 * kappa * ||b||.
"""
import numpy as np
import pytest
import torch

from gpu_util import rel, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


def _small_stream(count, rate, seed):
    from paper_2508_14209_amd import serve
    return serve.make_requests(count, rate, seed=seed, d_lo=1 << 12, d_hi=1 << 15,
                               ns=(8, 16, 32), nrhs_max=4, kappa_lo=1e1, kappa_hi=1e3)


def test_serving_stream_alone_vs_mix(ms, orc):
    from paper_2508_14209_amd import serve
    reqs = _small_stream(48, 4000.0, seed=3)
    srv = serve.Server(hbm_budget=1 << 30, max_inflight=16, max_batch=8, streams=3)
    for r in reqs:
        r.extra["kept"] = True
    done = srv.run(reqs, keep_tensors=True)
    assert len(done) == len(reqs) and all(r.status == ms.MS_OK for r in done)
    assert srv.nbatches > 1
    assert srv.admission.peak_bytes <= (1 << 30) or srv.admission.count == 0
    for i, r in enumerate(sorted(done, key=lambda q: q.id)):
        T = r.tensors
        Xmix = to_host(T["X"])
        Xa, ws = ms.sketch_lstsq(T["A"], T["B"], T["h"], T["s"], T["G"], T["k"])
        ms.check_status(ws)
        Xal = to_host(Xa)
        assert rel(Xmix, Xal) <= 1e-5 * r.kappa, (r.id, rel(Xmix, Xal), r.kappa)
        A = to_host(T["A"]).astype(np.float64)
        B = to_host(T["B"]).astype(np.float64)
        rm, ra = np.linalg.norm(B - A @ Xmix), np.linalg.norm(B - A @ Xal)
        assert abs(rm - ra) <= 1e-5 * r.kappa * np.linalg.norm(B)
        if i % 8 == 0:  # sampled requests against the oracle (same device inputs)
            Xr, _, _ = orc.sketch_lstsq(to_host(T["A"]), to_host(T["B"]), to_host(T["h"]),
                                        to_host(T["s"]), to_host(T["G"]).astype(np.float64),
                                        T["k"])
            assert rel(Xmix, Xr) <= 1e-5 * r.kappa


def test_serving_respects_hbm_budget(ms):
    from paper_2508_14209_amd import serve
    reqs = _small_stream(24, 0.0, seed=4)   # all arrive at once
    budget = 3 * max(serve.footprint_bytes(r.d, r.n, r.nrhs, r.k, r.k2) for r in reqs)
    srv = serve.Server(hbm_budget=budget, max_inflight=64, max_batch=8, streams=2)
    done = srv.run(reqs)
    assert len(done) == 24 and all(r.status == ms.MS_OK for r in done)
    assert srv.admission.peak_bytes <= budget
    assert srv.nbatches >= 3


@pytest.mark.parametrize("single", [True, False])
def test_serving_plain_fp64_paths(ms, orc, single):
    # the plain FP64 comparators of the serving measurement: A, B and G
    # promoted exactly to FP64, solved one request per sketch_lstsq call (the
    # paper's path) or in batches; every request against the oracle at the
    # FP64 bar on the same (promoted) inputs
    # (condition numbers up to 10, so the association-order differences stay
    # well inside the FP64 bar)
    from paper_2508_14209_amd import serve
    reqs = serve.make_requests(12, 4000.0, seed=5, d_lo=1 << 12, d_hi=1 << 15, ns=(8, 16, 32),
                               nrhs_max=4, kappa_lo=1.0, kappa_hi=10.0)
    for r in reqs:
        r.extra["kept"] = True
    srv = serve.Server(hbm_budget=1 << 30, max_inflight=16, max_batch=4, streams=2,
                       g_dtype="f64", a_dtype="f64", single=single)
    done = srv.run(reqs, keep_tensors=True)
    assert len(done) == len(reqs) and all(r.status == ms.MS_OK for r in done)
    if single:
        assert srv.nbatches == len(reqs)
    for r in done:
        T = r.tensors
        assert T["A"].dtype == torch.float64 and T["G"].dtype == torch.float64
        Xr, _, _ = orc.sketch_lstsq(to_host(T["A"]), to_host(T["B"]), to_host(T["h"]),
                                    to_host(T["s"]), to_host(T["G"]), T["k"])
        assert rel(to_host(T["X"]), Xr) <= 1e-12, (r.id, single)


def test_serving_default_stream_mixed_precision(ms, orc):
    # Requests drawn from the serving workload as specified (d log-uniform in
    # [2^14, 2^20], n in {8, ..., 128}, 1-8 right-hand sides, kappa
    # log-uniform in [1e1, 1e5], A = Z diag Q in FP32 with Q orthogonal),
    # solved on the path the serving measurement runs: batched, FP32 sketch,
    # BF16 Gaussian stage (three exact BF16 terms of the sketch), FP64 QR and
    # two FP64-residual refinement steps, by one persistent runner per solver
    # stream replaying its captured launch sequence (batches padded to the
    # runner's count); in the mix and each alone.
    # Checks per request:
    #  * against the oracle's FP64 sketch-and-solve with the same (h, s, G):
    #    the refinement's fixed point satisfies Q~^T G C (b - A x) = 0 with Q~
    #    from the FP32 sketch, whose rounding E (~u32 ||S A||) moves x by
    #    (S A)^+ ... E^T r_s: relative to ||x||, at most about kappa^2 u32 eta
    #    with eta = ||b - A x|| / (||A|| ||x||) (the scaled residual); bar
    #    2 kappa^2 u32 eta (never below 1e-8);
    #  * mix vs alone: the same iteration from FP32 sketches that differ only
    #    in association order, each within that bound of the FP64 solution:
    #    bar twice it;
    #  * the residual ratio rho against LAPACK's FP64 optimum: the mixed
    #    result's rho within 1% of the FP64 sketch-and-solve's (same sketch,
    #    so the same distortion); the fraction with rho <= 2 and the largest
    #    rho are reported (small n has a tail above 2 by the embedding's
    #    distortion itself, not by the precision).
    from paper_2508_14209_amd import serve
    reqs = serve.make_requests(16, 2000.0, seed=21)
    for r in reqs:
        r.extra["kept"] = True
    srv = serve.Server(hbm_budget=32 << 30, max_inflight=64, max_batch=8, streams=3,
                       g_dtype="bf16", refine_steps=2, persistent=True)
    srv.warm_runners(serve.make_requests(4, 0.0, seed=22))
    done = srv.run(reqs, keep_tensors=True)
    assert len(srv.runners) == 3 and all(r.graph is not None for r in srv.runners.values())
    assert len(done) == len(reqs) and all(r.status == ms.MS_OK for r in done)
    rhos, rhos64 = [], []
    for r in sorted(done, key=lambda q: q.id):
        T = r.tensors
        Xmix = to_host(T["X"])
        Xa, ws = ms.sketch_lstsq(T["A"], T["B"], T["h"], T["s"], T["G"], T["k"], refine_steps=2)
        ms.check_status(ws)
        Xal = to_host(Xa)
        A64 = to_host(T["A"]).astype(np.float64)
        B64 = to_host(T["B"]).astype(np.float64)
        G64 = to_host(T["G"].float()).astype(np.float64)
        X64, _, _ = orc.sketch_lstsq(A64, B64, to_host(T["h"]), to_host(T["s"]), G64, T["k"])
        xo = np.linalg.lstsq(A64, B64, rcond=None)[0]
        ro = np.linalg.norm(B64 - A64 @ xo)
        rho = np.linalg.norm(B64 - A64 @ Xmix) / ro
        rho64 = np.linalg.norm(B64 - A64 @ X64) / ro
        e_mix_alone, e_64 = rel(Xmix, Xal), rel(Xmix, X64)
        sv = np.linalg.svd(A64.T @ A64, compute_uv=False)
        kap = float(np.sqrt(sv[0] / sv[-1]))
        eta = float(np.linalg.norm(B64 - A64 @ X64) / (np.sqrt(sv[0]) * np.linalg.norm(X64)))
        bar = max(1e-8, 2 * kap ** 2 * 2.0 ** -24 * eta)
        print("req %2d d=%7d n=%3d nrhs=%d kappa=%.1e: mix-alone %.2e  vs FP64 s&s %.2e "
              "(bar %.1e)  rho %.4f (FP64 s&s %.4f)"
              % (r.id, r.d, r.n, r.nrhs, kap, e_mix_alone, e_64, bar, rho, rho64), flush=True)
        assert e_64 <= bar, r.id
        assert e_mix_alone <= 2 * bar, r.id
        assert abs(rho - rho64) <= 0.01 * rho64, r.id
        rhos.append(rho)
        rhos64.append(rho64)
        T.clear()
    rhos = np.array(rhos)
    print("fraction rho <= 2: %.3f, max rho %.3f (FP64 sketch-and-solve: %.3f, %.3f)"
          % (np.mean(rhos <= 2), rhos.max(), np.mean(np.array(rhos64) <= 2), max(rhos64)))


def test_serving_deterministic_alone_equals_mix_bit_for_bit(ms):
    # deterministic serving: persistent runners replaying captured graphs,
    # BF16 Gaussian stage, one refinement step; each request's X equals, bit
    # for bit, the X of the same request solved in a batch of its own
    from paper_2508_14209_amd import serve
    reqs = serve.make_requests(40, 4000.0, seed=21, d_lo=1 << 12, d_hi=1 << 16,
                               ns=(8, 16, 32, 64), nrhs_max=4, kappa_lo=1e1, kappa_hi=1e5)
    for r in reqs:
        r.extra["kept"] = True
    srv = serve.Server(hbm_budget=8 << 30, max_inflight=32, max_batch=8, streams=3,
                       g_dtype="bf16", refine_steps=1, persistent=True, graphs=True,
                       deterministic=True, max_shape=(1 << 16, 64, 4))
    srv.warm_runners(reqs[:8])
    done = srv.run(reqs, keep_tensors=True)
    assert len(done) == len(reqs) and all(r.status == ms.MS_OK for r in done)
    assert srv.nbatches > 1
    for r in sorted(done, key=lambda q: q.id):
        T = r.tensors
        Xmix = to_host(T["X"]).copy()
        alone = dict(T)
        alone["X"] = ms.empty_colmajor(r.n, r.nrhs, torch.float64, "cuda")
        run = ms.sketch_lstsq_batched([alone], refine_steps=1, deterministic=True)
        assert run.status()[0] == ms.MS_OK
        torch.cuda.synchronize()
        assert np.array_equal(to_host(alone["X"]), Xmix), r.id
