"""Host-only checks of the serving loop's admission policy and request
stream (no GPU)."""
import numpy as np

import synth


def test_admission_budget_and_slots():
    from paper_2508_14209_amd.serve import Admission
    a = Admission(hbm_budget=100, max_inflight=3)
    assert a.try_admit(60)
    assert not a.try_admit(50)          # would exceed the budget
    assert a.try_admit(40)
    assert not a.try_admit(1)           # budget full
    a.release(60)
    assert a.try_admit(10) and a.try_admit(10)
    assert not a.try_admit(1)           # three slots in use
    assert a.peak_bytes <= 100
    b = Admission(hbm_budget=10, max_inflight=4)
    assert b.try_admit(500)             # larger than the budget: admitted alone
    assert not b.try_admit(1)
    b.release(500)
    assert b.try_admit(1)


def test_request_stream_distribution():
    reqs = synth.serving_requests(4096, seed=1)
    d = np.array([r["d"] for r in reqs])
    n = np.array([r["n"] for r in reqs])
    nrhs = np.array([r["nrhs"] for r in reqs])
    kap = np.array([r["kappa"] for r in reqs])
    assert d.min() >= 2 ** 14 and d.max() <= 2 ** 20
    assert abs(np.log2(d).mean() - 17.0) < 0.15          # log-uniform on [14, 20]
    assert set(n.tolist()) == {8, 16, 32, 64, 128}
    assert set(nrhs.tolist()) == set(range(1, 9))
    assert kap.min() >= 10 and kap.max() <= 1e5
    assert all(r["k"] == 2 * r["n"] ** 2 and r["k2"] == 2 * r["n"] for r in reqs)
    t = synth.poisson_arrivals(4096, 2000.0, seed=1)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 2000.0) < 4 * (1 / 2000.0) / np.sqrt(4096)
    assert np.all(gaps >= 0)
