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
