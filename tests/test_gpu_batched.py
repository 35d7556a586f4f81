"""GPU parity of the batched multisketch sketch-and-solve: every problem of a
mixed batch against the oracle, each result the same alone and in the mix,
HIP-graph capture and replay with rewritten descriptors, per-problem errors.

Bar: FP64 problems 1e-12 normwise relative against the oracle (and against
the same problem solved alone); FP32 problems 1e-5 (well-conditioned, FP32
sketch, against the exact-sum FP32 sketch); BF16 Gaussian stage against the
oracle's BF16 path 1e-2 (the sketch's last-bit differences may move entries
across a BF16 rounding boundary, each such entry changing by 2^-8 relative).
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


def make_problem(ms, d, n, nrhs, seed, dtype=np.float64, gd="f64", noise=1e-6):
    k, k2 = 2 * n * n, 2 * n
    A = synth.normal_matrix(d, n, seed=seed, dtype=dtype)
    B, _ = synth.lstsq_rhs(A, nrhs, seed=seed, noise=noise)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype=gd)
    host = dict(A=A, B=B, h=h, s=s, G=G, k=k)
    dev = dict(A=to_dev(A), B=to_dev(B), h=to_dev(h), s=to_dev(s),
               G=bf16_dev(G) if gd == "bf16" else to_dev(G), k=k,
               X=ms.empty_colmajor(n, nrhs, torch.float64, "cuda"))
    return host, dev


SHAPES = [(5000, 4, 1), (20000, 8, 3), (70001, 16, 2), (3000, 16, 8), (40000, 32, 1),
          (100, 8, 1), (65536, 64, 4), (30000, 128, 1)]


def test_batched_fp64_mixed_matches_oracle_and_alone(ms, orc):
    probs = [make_problem(ms, d, n, r, seed=100 + i) for i, (d, n, r) in enumerate(SHAPES)]
    runner = ms.sketch_lstsq_batched([p[1] for p in probs])
    st, per = runner.status()
    assert st == ms.MS_OK and all(v == ms.MS_OK for v in per)
    for (host, dev), (d, n, r) in zip(probs, SHAPES):
        Xb = to_host(dev["X"])
        Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"], host["G"], host["k"])
        assert rel(Xb, Xr) <= 1e-12, (d, n, r, rel(Xb, Xr))
        Xa, ws = ms.sketch_lstsq(dev["A"], dev["B"], dev["h"], dev["s"], dev["G"], host["k"])
        ms.check_status(ws)
        assert rel(Xb, to_host(Xa)) <= 1e-12


@pytest.mark.parametrize("gd", ["f32", "bf16"])
def test_batched_fp32(ms, orc, gd):
    shapes = [(30000, 8, 2), (50000, 16, 1), (20000, 32, 4)]
    probs = [make_problem(ms, d, n, r, seed=200 + i, dtype=np.float32, gd=gd)
             for i, (d, n, r) in enumerate(shapes)]
    runner = ms.sketch_lstsq_batched([p[1] for p in probs])
    st, per = runner.status()
    assert st == ms.MS_OK
    for host, dev in probs:
        # reference sketch: Def. 3's exact sums rounded once to FP32 (the
        # batched kernel sums each item's rows in FP64); the BF16 Gaussian
        # stage takes the sketch as three BF16 terms that sum to it exactly
        # (the default), so both G dtypes meet the FP32 bar
        Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"], host["G"],
                                    host["k"], y_acc64=True)
        err = rel(to_host(dev["X"]), Xr)
        print(gd, host["A"].shape, "err %.3e" % err)
        assert err <= 1e-5


def test_batched_graph_replay_with_new_problems(ms, orc):
    # n = 32 (33 columns in 9 column tiles) packs its rows into bucket words;
    # the second set has more rows than the captured capacity, so its replays
    # read h and s in every work item instead
    shapes = [(20000, 8, 2), (30000, 16, 1), (10000, 8, 3), (12000, 32, 1)]
    set1 = [make_problem(ms, d, n, r, seed=300 + i) for i, (d, n, r) in enumerate(shapes)]
    set2 = [make_problem(ms, d + 777, n, r, seed=400 + i) for i, (d, n, r) in enumerate(shapes)]
    runner = ms.BatchRunner([p[1] for p in set1])
    runner.capture()
    for rep in range(3):
        for which in (set1, set2):
            runner.set_problems([p[1] for p in which])
            for _, dev in which:
                dev["X"].fill_(float("nan"))
            runner.replay()
            torch.cuda.synchronize()
            # eager work between replays
            torch.ones(1024, device="cuda").sum().item()
            st, per = runner.status()
            assert st == ms.MS_OK, (rep, st, per)
            for host, dev in which:
                Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"],
                                            host["G"], host["k"])
                assert rel(to_host(dev["X"]), Xr) <= 1e-12


def test_batched_pipelined_set_problems_without_host_sync(ms, orc):
    # set_problems(set1), replay, set_problems(set2), replay, ... enqueued back
    # to back with no host synchronisation: each replay must solve the set
    # whose descriptors were written just before it (the staging buffer of a
    # pending descriptor copy is not rewritten before that copy has run)
    shapes = [(20000, 8, 2), (30000, 16, 1), (12000, 32, 1)]
    sets = [[make_problem(ms, d + 101 * j, n, r, seed=800 + 10 * j + i)
             for i, (d, n, r) in enumerate(shapes)] for j in range(4)]
    runner = ms.BatchRunner([p[1] for p in sets[0]])
    runner.capture()
    for which in sets:
        for _, dev in which:
            dev["X"].fill_(float("nan"))
    torch.cuda.synchronize()
    for which in sets:
        runner.set_problems([p[1] for p in which])
        runner.replay()
    torch.cuda.synchronize()
    st, per = runner.status()
    assert st == ms.MS_OK, (st, per)
    for j, which in enumerate(sets):
        for host, dev in which:
            Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"], host["G"],
                                        host["k"])
            assert rel(to_host(dev["X"]), Xr) <= 1e-12, j


def test_batched_per_problem_range_error(ms, orc):
    probs = [make_problem(ms, 5000, 8, 1, seed=500 + i) for i in range(3)]
    bad_h = probs[1][0]["h"].copy()
    bad_h[17] = probs[1][0]["k"]  # out of range
    probs[1][1]["h"] = to_dev(bad_h)
    runner = ms.sketch_lstsq_batched([p[1] for p in probs])
    st, per = runner.status()
    assert st == ms.MS_ERR_RANGE
    assert per == [ms.MS_OK, ms.MS_ERR_RANGE, ms.MS_OK]
    for i in (0, 2):
        host, dev = probs[i]
        Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"], host["G"], host["k"])
        assert rel(to_host(dev["X"]), Xr) <= 1e-12


def test_batched_replay_larger_than_capacity_is_refused(ms):
    small = [make_problem(ms, 4000, 8, 1, seed=600 + i) for i in range(2)]
    big = [make_problem(ms, 4000, 16, 1, seed=700 + i) for i in range(2)]
    runner = ms.BatchRunner([p[1] for p in small])
    runner.set_problems([p[1] for p in big])
    runner.launch()
    st, per = runner.status()
    assert st == ms.MS_ERR_NOMEM and per == [ms.MS_ERR_NOMEM] * 2


def make_scaled_problem(ms, d, n, nrhs, seed, gd="bf16", decades=4.0):
    """FP32 A = Z diag(logspace(0, -decades, n)), BF16 (or FP32) Gaussian stage."""
    k, k2 = 2 * n * n, 2 * n
    Z = synth.normal_matrix(d, n, seed=seed, dtype=np.float64)
    A = np.asfortranarray((Z * np.logspace(0, -decades, n)[None, :]).astype(np.float32))
    B, _ = synth.lstsq_rhs(A, nrhs, seed=seed)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed, dtype=gd)
    host = dict(A=A, B=B, h=h, s=s, G=G, k=k)
    dev = dict(A=to_dev(A), B=to_dev(B), h=to_dev(h), s=to_dev(s),
               G=bf16_dev(G) if gd == "bf16" else to_dev(G), k=k,
               X=ms.empty_colmajor(n, nrhs, torch.float64, "cuda"))
    return host, dev


REFINE_SHAPES = [(1 << 17, 8, 1), (100003, 16, 4), (1 << 16, 32, 8)]


@pytest.mark.parametrize("yt", [1, 3])
@pytest.mark.parametrize("refine", [0, 1, 2, 3])
def test_batched_bf16_refinement(ms, orc, refine, yt):
    # Mixed precision in one batched call: FP32 CountSketch, BF16 Gaussian
    # stage, FP64 QR, then FP64-residual refinement steps per problem.  Each
    # X's error against the FP64 sketch-and-solve solution for the same
    # (h, s, G) (oracle) must equal, to association-order effects, the error
    # of the single-problem path at the same step count (whose contraction is
    # pinned against the oracle's own iteration elsewhere); and three steps
    # must have removed the BF16 error (O(1) without refinement; each step
    # contracts it by about u_bf16 times the conditioning of the
    # column-equilibrated sketch, ~1e-2 for k2 = 2n).
    probs = [make_scaled_problem(ms, d, n, r, seed=800 + i)
             for i, (d, n, r) in enumerate(REFINE_SHAPES)]
    runner = ms.sketch_lstsq_batched([p[1] for p in probs], refine_steps=refine, y_terms=yt)
    st, per = runner.status()
    assert st == ms.MS_OK and all(v == ms.MS_OK for v in per)
    for (host, dev), shape in zip(probs, REFINE_SHAPES):
        Xb = to_host(dev["X"])
        A64, B64 = host["A"].astype(np.float64), host["B"].astype(np.float64)
        X64, _, _ = orc.sketch_lstsq(A64, B64, host["h"], host["s"],
                                     host["G"].astype(np.float64), host["k"])
        err = rel(Xb, X64)
        Xa, ws = ms.sketch_lstsq(dev["A"], dev["B"], dev["h"], dev["s"], dev["G"], host["k"],
                                 refine_steps=refine, y_terms=yt)
        ms.check_status(ws)
        ea = rel(to_host(Xa), X64)
        print(shape, "y_terms=%d refine=%d batched %.3e alone %.3e" % (yt, refine, err, ea))
        # One BF16 term: the error starts at O(1) and each step contracts
        # it by c ~ u_bf16 times the conditioning of the column-equilibrated
        # sketch (1e-2 or less here: e_1 / e_0 measured 1e-2 for n = 8, 2e-3
        # for n = 32) down to the fixed point's offset (a few 1e-6): bounds
        # 5, 5e-2, 1e-4, 1e-5 after 0..3 steps; both paths round the same
        # sketch values to BF16 and agree to the last digits.  Three exact
        # terms: only the FP32 sketch's rounding remains (a few 1e-4 before,
        # ~1e-10 after one step); the batched and single sketches differ in
        # association order, so only the bound is checked.
        bound = ({0: 5.0, 1: 5e-2, 2: 1e-4, 3: 1e-5} if yt == 1 else
                 {0: 1e-2, 1: 1e-8, 2: 1e-8, 3: 1e-8})[refine]
        assert np.isfinite(Xb).all() and err <= bound, (shape, err)
        if yt == 1:
            assert err <= 1.2 * ea + 1e-7, (shape, err, ea)


def test_batched_fp64_refinement_keeps_parity(ms, orc):
    # FP64 throughout: the first pass already is the sketch-and-solve
    # solution to rounding, so refinement steps leave it within 1e-12.
    shapes = [(20000, 8, 2), (30001, 16, 1)]
    probs = [make_problem(ms, d, n, r, seed=900 + i) for i, (d, n, r) in enumerate(shapes)]
    runner = ms.sketch_lstsq_batched([p[1] for p in probs], refine_steps=2)
    st, per = runner.status()
    assert st == ms.MS_OK
    for host, dev in probs:
        Xr, _, _ = orc.sketch_lstsq(host["A"], host["B"], host["h"], host["s"], host["G"], host["k"])
        assert rel(to_host(dev["X"]), Xr) <= 1e-12


def test_batched_refinement_graph_replay(ms, orc):
    # the refinement launches are captured with the rest; replays with new
    # descriptors (same count, no larger) reproduce the eager results
    set1 = [make_scaled_problem(ms, d, n, r, seed=1000 + i)
            for i, (d, n, r) in enumerate([(40000, 8, 2), (30000, 16, 1)])]
    set2 = [make_scaled_problem(ms, d, n, r, seed=1100 + i)
            for i, (d, n, r) in enumerate([(35000, 8, 2), (20000, 16, 1)])]
    eager = {}
    for name, which in (("1", set1), ("2", set2)):
        r = ms.sketch_lstsq_batched([p[1] for p in which], refine_steps=2)
        assert r.status()[0] == ms.MS_OK
        eager[name] = [to_host(p[1]["X"]).copy() for p in which]
    runner = ms.BatchRunner([p[1] for p in set1], refine_steps=2)
    runner.capture()
    for rep in range(3):
        for name, which in (("1", set1), ("2", set2)):
            runner.set_problems([p[1] for p in which])
            for _, dev in which:
                dev["X"].fill_(float("nan"))
            runner.replay()
            torch.cuda.synchronize()
            torch.ones(1024, device="cuda").sum().item()
            st, per = runner.status()
            assert st == ms.MS_OK, (rep, st, per)
            for (host, dev), Xe in zip(which, eager[name]):
                assert rel(to_host(dev["X"]), Xe) <= 1e-6, (rep, name)


# ------------------------------------------------------------------ deterministic mode
@pytest.mark.parametrize("refine", [0, 1])
def test_batched_deterministic_alone_vs_mix_bit_identical(ms, orc, refine):
    # the deterministic batched CountSketch folds every bucket in row order,
    # and every other stage of a problem depends on that problem alone: its X
    # is the same bit for bit in any batch (here: the whole mix, the mix
    # reversed, and a batch of its own)
    specs = [(70001, 8, 3, 1, "bf16"), (4097, 16, 1, 2, "bf16"), (123457, 32, 4, 3, "bf16"),
             (30000, 8, 2, 4, "bf16"), (65536, 64, 1, 5, "bf16"), (9000, 16, 8, 6, "bf16")]
    hosts, devs = [], []
    for d, n, nrhs, seed, gd in specs:
        hst, dv = make_problem(ms, d, n, nrhs, seed=seed + 40, dtype=np.float32, gd=gd)
        hosts.append(hst)
        devs.append(dv)
    print("deterministic batch refine=%d" % refine, flush=True)
    ms.sketch_lstsq_batched(devs, refine_steps=refine, deterministic=True)
    torch.cuda.synchronize()
    X_mix = [to_host(p["X"]).copy() for p in devs]
    for p in devs:
        p["X"].fill_(np.nan)
    ms.sketch_lstsq_batched(devs[::-1], refine_steps=refine, deterministic=True)
    torch.cuda.synchronize()
    X_rev = [to_host(p["X"]).copy() for p in devs]
    for i, p in enumerate(devs):
        p["X"].fill_(np.nan)
        r = ms.sketch_lstsq_batched([p], refine_steps=refine, deterministic=True)
        assert r.status()[0] == ms.MS_OK
        torch.cuda.synchronize()
        Xa = to_host(p["X"])
        assert np.array_equal(Xa, X_mix[i]) and np.array_equal(Xa, X_rev[i]), i
    # and the solutions are the problems' sketch-and-solve solutions: the
    # FP32 sketch is the oracle's sequential FP32 fold exactly, the BF16
    # stage takes it as three exact terms (FP32 accumulation): against the
    # oracle's FP32-sketch path with FP64 Gaussian stage, 1e-5 at refine 0
    # (well-conditioned N(0,1) data); with a step, against FP64
    # sketch-and-solve of the promoted data at 1e-5
    for i, hst in enumerate(hosts):
        if refine == 0:
            Xr, _, _ = orc.sketch_lstsq(hst["A"], hst["B"], hst["h"], hst["s"],
                                        hst["G"].astype(np.float64), hst["k"])
        else:
            Xr, _, _ = orc.sketch_lstsq(hst["A"].astype(np.float64), hst["B"].astype(np.float64),
                                        hst["h"], hst["s"], hst["G"].astype(np.float64), hst["k"])
        assert rel(X_mix[i], Xr) <= 1e-5, (i, rel(X_mix[i], Xr))


def test_batched_deterministic_fp64_matches_oracle(ms, orc):
    # FP64 data: the sorted fold is the oracle's FP64 fold bit for bit; the
    # FP64 Gaussian stage (K split in fixed chunks, partials summed in order)
    # and QR keep the FP64 bar
    hst, dv = make_problem(ms, 50001, 16, 2, seed=77)
    hst2, dv2 = make_problem(ms, 3000, 8, 1, seed=78)
    ms.sketch_lstsq_batched([dv, dv2], deterministic=True)
    torch.cuda.synchronize()
    for h_, d_ in ((hst, dv), (hst2, dv2)):
        Xr, _, _ = orc.sketch_lstsq(h_["A"], h_["B"], h_["h"], h_["s"], h_["G"], h_["k"])
        assert rel(to_host(d_["X"]), Xr) <= 1e-12


def test_batched_refinement_early_stop(ms, orc):
    # refine_tol_log2 = x: a problem stops refining once a step's correction
    # is at most 2^-x of its X.  x = 1 stops every problem after its first
    # step (the first correction is far below half of X): the result is that
    # of one step, bit for bit (deterministic mode, so that the two runs see
    # the same arithmetic).  x = 60 stops none: the result is that of all
    # steps, bit for bit.
    probs = []
    for i, (d, n, nrhs) in enumerate([(40001, 8, 2), (70000, 16, 1), (9000, 32, 4)]):
        _, dv = make_problem(ms, d, n, nrhs, seed=90 + i, dtype=np.float32, gd="bf16")
        probs.append(dv)

    def run(steps, tol):
        for p in probs:
            p["X"].fill_(np.nan)
        r = ms.sketch_lstsq_batched(probs, refine_steps=steps, deterministic=True,
                                    refine_tol_log2=tol)
        assert r.status()[0] == ms.MS_OK
        torch.cuda.synchronize()
        return [to_host(p["X"]).copy() for p in probs]

    one, three = run(1, 0), run(3, 0)
    stop1, stop60 = run(3, 1), run(3, 60)
    for a, b in zip(one, stop1):
        assert np.array_equal(a, b)
    for a, b in zip(three, stop60):
        assert np.array_equal(a, b)
