"""The autotuner on the GPU: it times the CountSketch and batched-solve
variants, keeps only candidates whose results agree with the default, caches
the fastest, and the cached choice reproduces the oracle's result."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture()
def at(tmp_path, monkeypatch):
    monkeypatch.setenv("MSKETCH_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2508_14209_amd import autotune
    return autotune


def test_tune_countsketch_choice_matches_oracle(at, orc):
    import paper_2508_14209_amd as ms
    d, n, k = 200000, 8, 1024
    A = synth.normal_matrix(d, n, seed=41)
    h = synth.bucket_map(d, k, seed=41)
    s = synth.signs(d, seed=41)
    Ad, hd, sd = to_dev(A), to_dev(h), to_dev(s)
    best = at.tune_countsketch(Ad, hd, sd, k, reps=2)
    assert best["candidates"] >= 2 and best["ms"] > 0
    cols, sched = at.lookup_countsketch(d, n, k, Ad.dtype)
    assert (cols, sched) == (best["tile_cols"], best["schedule"])
    code, _ = ms.pack_sketch(hd, sd, k)
    Y = ms.empty_colmajor(k, n, torch.float64, "cuda")
    Y.zero_()
    ws = ms.workspace(256, "cuda")
    ms.countsketch_accumulate(Ad, code, k, Y, ws=ws, tile_cols=cols, schedule=sched)
    ms.check_status(ws)
    assert rel(to_host(Y), orc.countsketch(A, h, s, k)) <= 1e-12


def test_tune_batch_choice_matches_oracle(at, orc):
    import paper_2508_14209_amd as ms
    shapes = [(30000, 8, 2), (50000, 16, 1), (20000, 8, 3)]
    probs = []
    for i, (d, n, r) in enumerate(shapes):
        k, k2 = 2 * n * n, 2 * n
        A = synth.normal_matrix(d, n, seed=50 + i)
        B, _ = synth.lstsq_rhs(A, r, seed=50 + i)
        h = synth.bucket_map(d, k, seed=50 + i)
        s = synth.signs(d, seed=50 + i)
        G = synth.gaussian_sketch(k2, k, seed=50 + i)
        probs.append((dict(A=A, B=B, h=h, s=s, G=G, k=k),
                      dict(A=to_dev(A), B=to_dev(B), h=to_dev(h), s=to_dev(s), G=to_dev(G), k=k,
                           X=ms.empty_colmajor(n, r, torch.float64, "cuda"))))
    dev = [p[1] for p in probs]
    best = at.tune_batch(dev, reps=1, rows=(13, 15), kchunks=(5, 8))
    assert best["candidates"] >= 2
    rl, kl = at.batch_params(dev)
    assert (rl, kl) == (best["rows_log2"], best["kchunk_log2"])
    for _, dv in probs:
        dv["X"].fill_(float("nan"))
    r = ms.BatchRunner(dev, rows_log2=rl, kchunk_log2=kl)
    r.launch()
    assert r.status()[0] == ms.MS_OK
    for host, dv in probs:
        Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"], host["G"],
                                    host["k"])
        assert rel(to_host(dv["X"]), Xr) <= 1e-12
