#!/usr/bin/env python3
"""Benchmark of the multisketch sketch-and-solve least-squares hot path on one GPU.

One step = one full multisketch sketch-and-solve (Alg. 1 with S = G C) of the
FP64 workload
    A 4,194,304 x 64 i.i.d. N(0,1), b = A x* + 1e-6 N(0,1) (one right-hand side),
    CountSketch k = 8192, Gaussian stage G 128 x 8192 with N(0, 1/128) entries,
    Householder QR of the 128 x 64 sketch, Q^T b, triangular solve,
run by ``sketch_lstsq`` through the C ABI with every input resident in HBM.

Also measured, each over its own timed loop on the launch stream:
  * the dominant kernel -- the LDS-binned CountSketch of [A | b]
    (``countsketch_accumulate``, one kernel per call) -- for the roofline;
  * the global-atomic CountSketch (the Alg. 2 baseline) and the deterministic
    sorted CountSketch, for comparison;
  * the Gaussian stage alone (matrix cores, FP64);
  * the CPU oracle on the host, for the cpu_baseline entry;
  * the continuous-batching serving loop over a stream of uneven requests
    (open loop at 2,000/s and closed loop), p50/p99 latency and solves/s;
  * a batch of such problems solved by the plain FP64 path one by one and by
    the batched mixed-precision path (BF16 Gaussian stage, FP64 QR and
    refinement), with solves/s and residual ratios against the FP64 QR optimum.

Prints ONE JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 matrix/vector, published
METRIC = "CountSketch GB/s & % HBM peak; multisketch LS solves/s + p99 latency"
WORKLOAD = "multisketch_lstsq_4194304x64_f64_k8192_k2_128"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", default="lds", choices=["lds", "atomic", "sorted"])
    ap.add_argument("--seed", type=int, default=14209)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle baseline (0 disables it)")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the serving stream legs (0 skips them)")
    ap.add_argument("--compare-problems", type=int, default=64,
                    help="problems of the batched mixed-precision vs plain FP64 leg (0 skips it)")
    ap.add_argument("--other-configs", type=int, default=1,
                    help="also time the FP32 16,777,216 x 128 and the mixed-precision "
                         "8,388,608 x 256 solves (0 skips them)")
    ap.add_argument("--extras", type=int, default=1,
                    help="1: also measure rand_cholQR / normal equations, the SRHT and the "
                         "hash-generated CountSketch (0 skips them, e.g. to profile the headline "
                         "solve alone)")
    ap.add_argument("--refine", type=int, default=2,
                    help="FP64-residual refinement steps of the mixed-precision legs")
    ap.add_argument("--only", default=None,
                    choices=["countsketch", "countsketch_f32_k32768", "countsketch_f32_k131072",
                             "copy", "gaussian_f64", "gaussian_bf16", "batched_mixed",
                             "solve_fp32", "solve_mixed", "rand_cholqr",
                             "normal_equations", "countsketch_hashed", "srht",
                             "paper_comparison", "countsketch_sorted", "batched_fp64"],
                    help="profiling runs: launch only the LDS CountSketch of [A | b] (--steps "
                         "times), only a plain device copy of 1 GiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters), or only the Gaussian stage of the "
                         "FP64 workload (128 x 8192 times 8192 x 65) or of the mixed-precision "
                         "workload (BF16 512 x 131,072 times 131,072 x 260); prints a short "
                         "JSON line")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles",
                               "k_cs_lds_xcd_multisketch_lstsq_4194304x65_f64_traffic.md")


def measured_traffic():
    """HBM bytes per CountSketch launch from the committed counter profile,
    or None once the kernel's source differs from the profiled one."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m_t = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    m_h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not (m_t and m_h):
        return None
    return int(m_t.group(1)) if countsketch_source_hash() == m_h.group(1) else None


def countsketch_source_hash():
    """sha256 of the single-problem CountSketch sources: countsketch.hip up
    to its batched section and ms_internal.h up to the rand_cholQR
    declarations (what follows there is not used by the profiled kernel)."""
    import hashlib
    h = hashlib.sha256()
    for f, mark in (("countsketch.hip", "// " + "-" * 66 + " batched"),
                    ("ms_internal.h", "// rand_cholQR least squares (randcholqr.hip)")):
        with open(os.path.join(ROOT, "paper_2508_14209_amd", "csrc", f)) as fh:
            text = fh.read()
        h.update(text[:text.index(mark)].encode())
    return h.hexdigest()


def event_pair(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


SERVE_WORKLOAD = ("Poisson arrivals at 2,000/s; d log-uniform in [2^14, 2^20], n uniform in "
                  "{8,16,32,64,128}, 1-8 right-hand sides, FP32 A = N(0,1) diag(logspace(0, "
                  "-log10 kappa, n)), kappa log-uniform in [1e1, 1e5]; k = 2n^2, k2 = 2n")


def serving_leg(ms, torch, np, count, seed, refine, dev):
    """Continuous-batching serving loop over the request stream: open loop at
    2,000 requests/s and closed loop (all requests at t = 0, saturation), for
    the mixed-precision batched solver with `refine` steps (top-level keys)
    and, under "variants", for every path: the plain FP64 multisketch one
    request per call (the paper's path) and batched, and the mixed-precision
    batched solver with 0..3 refinement steps."""
    from paper_2508_14209_amd import serve
    out = {"workload": SERVE_WORKLOAD, "requests": count, "g_dtype": "bf16",
           "refine_steps": refine, "max_batch": 64, "streams": 4}

    xopt = {}   # request id -> (x_opt, ||B - A x_opt||), FP64 on the device

    def rho_stats(done):
        """Residual ratio rho = ||B - A X|| / ||B - A x_opt|| (Frobenius over
        the right-hand sides) of the sampled requests; x_opt from a library
        FP64 QR least-squares solve on the device (measurement only)."""
        rhos = []
        for r in done:
            T = r.tensors
            if T is None or r.status != ms.MS_OK:
                continue
            A = T["A"].double()
            B = T["B"].double()
            if r.id not in xopt:
                xo = torch.linalg.lstsq(A, B).solution
                xopt[r.id] = (B - A @ xo).norm().item()
            rhos.append((B - A @ T["X"]).norm().item() / xopt[r.id])
            r.tensors = None
        rhos = np.array(rhos)
        return {"sampled": int(rhos.size), "fraction_le_2": float(np.mean(rhos <= 2.0)),
                "p50": float(np.percentile(rhos, 50)), "p99": float(np.percentile(rhos, 99)),
                "max": float(rhos.max())}

    def run_variant(g_dtype, a_dtype, single, rsteps, persistent=True):
        # each variant starts from an empty allocator cache: the previous
        # variant's closed loop leaves tens of GB of blocks of other sizes
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        # warm-up: load every kernel of the path once
        warm = serve.make_requests(16, 0.0, seed=seed + 7)
        serve.Server(max_batch=8, streams=2, g_dtype=g_dtype, a_dtype=a_dtype, single=single,
                     refine_steps=rsteps, device=dev).run(warm)
        res = {}
        for name, rate in (("open_loop_2000_per_s", 2000.0), ("closed_loop", 0.0)):
            if rate == 0.0:
                # an untimed closed loop first: the allocator then holds the
                # blocks of the loop's footprint (tens of GB), as a serving
                # process in steady state does, instead of mapping them during
                # the timed loop
                serve.Server(hbm_budget=96 << 30, max_inflight=512, max_batch=64,
                             streams=1 if single else 4, g_dtype=g_dtype, a_dtype=a_dtype,
                             single=single, refine_steps=rsteps, device=dev,
                             persistent=False).run(serve.make_requests(count, 0.0,
                                                                       seed=seed + 11))
            reqs = serve.make_requests(count, rate, seed=seed)
            if name.startswith("open"):
                for r in reqs[::32]:
                    r.extra["kept"] = True      # sampled for the residual ratio
            srv = serve.Server(hbm_budget=96 << 30, max_inflight=512, max_batch=64,
                               streams=1 if single else 4, g_dtype=g_dtype, a_dtype=a_dtype,
                               single=single, refine_steps=rsteps, device=dev,
                               persistent=persistent, tuned=True)
            if srv.persistent:
                srv.warm_runners(serve.make_requests(8, 0.0, seed=seed + 9))
            t0 = time.perf_counter()
            done = srv.run(reqs)
            wall = time.perf_counter() - t0
            summ = serve.summarize(done, wall)
            summ.update({"wall_s": wall, "batches": srv.nbatches,
                         "peak_inflight_bytes": srv.admission.peak_bytes,
                         "failed": sum(1 for r in done if r.status != ms.MS_OK)})
            if name.startswith("open"):
                summ["rho"] = rho_stats(done)
            res[name] = summ
            del srv, done
        return res

    main = run_variant("bf16", "f32", False, refine)
    out.update(main)
    variants = {"plain_fp64_one_per_call": run_variant("f64", "f64", True, 0),
                "plain_fp64_batched": run_variant("f64", "f64", False, 0)}
    for r in range(4):
        variants["mixed_bf16_batched_refine%d" % r] = (main if r == refine
                                                        else run_variant("bf16", "f32", False, r))
    variants["mixed_bf16_batched_refine%d_new_runner_per_batch" % refine] = run_variant(
        "bf16", "f32", False, refine, persistent=False)
    out["variants"] = variants
    out["runners"] = ("one persistent BatchRunner per solver stream (workspace sized once for "
                      "64 requests of 2^20 x 128 with 8 right-hand sides, batches padded with a "
                      "1-row placeholder), its launch sequence captured once in a graph and "
                      "replayed; batch tuning from the autotuner's cache when present")
    return out


def compare_problems(ms, torch, count, seed, dev):
    """A batch of serving-stream problems on the device, twice: FP64 A, B and
    G (the BF16 values promoted exactly) and FP32 A, B with BF16 G."""
    from paper_2508_14209_amd import serve
    reqs = serve.make_requests(count, 0.0, seed=seed)
    p64, pbf = [], []
    for r in reqs:
        t = serve.generate(r, dev, "f32")
        d, n, nrhs, k, k2 = r.d, r.n, r.nrhs, r.k, r.k2
        A64 = ms.empty_colmajor(d, n, torch.float64, dev)
        A64.copy_(t["A"])
        B64 = ms.empty_colmajor(d, nrhs, torch.float64, dev)
        B64.copy_(t["B"])
        Gb = torch.empty((k, k2), device=dev, dtype=torch.bfloat16).t()
        Gb.copy_(t["G"])
        G64 = ms.empty_colmajor(k2, k, torch.float64, dev)
        G64.copy_(Gb)                      # the BF16 values, exactly
        common = dict(h=t["h"], s=t["s"], k=k)
        p64.append(dict(A=A64, B=B64, G=G64, X=ms.empty_colmajor(n, nrhs, torch.float64, dev),
                        **common))
        pbf.append(dict(A=t["A"], B=t["B"], G=Gb, X=ms.empty_colmajor(n, nrhs, torch.float64, dev),
                        **common))
    return p64, pbf


def mixed_vs_fp64_leg(ms, torch, np, count, seed, refine, dev, reps=3):
    """The same batch of serving-stream problems solved (a) one by one by the
    plain FP64 multisketch path (A and G promoted exactly to FP64), (b) in
    one batched FP64 call, (c) in one batched mixed-precision call (FP32
    CountSketch, BF16 Gaussian stage, FP64 QR and `refine` FP64-residual
    refinement steps; the BF16 stage takes the sketch as three exact BF16
    terms) with 0, 1 and `refine` steps; solves/s of each and the residual
    ratio ||b - A x|| / ||b - A x_opt|| against the FP64 QR optimum x_opt
    (library QR in FP64 on the device, measurement only).  Headline: batched
    mixed over batched FP64 at the fewest refinement steps at which every
    problem's residual ratio is within max(2, its FP64 sketch-and-solve
    ratio) (1 + 1e-3)."""
    p64, pbf = compare_problems(ms, torch, count, seed, dev)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return count * reps / (time.perf_counter() - t0)

    wmax = max(ms.workspace_size("lstsq", d=p["A"].shape[0], n=p["A"].shape[1],
                                 nrhs=p["B"].shape[1], k=p["k"], k2=p["G"].shape[0])
               for p in p64)
    ws = ms.workspace(wmax, dev)

    def plain():
        for p in p64:
            ms.sketch_lstsq(p["A"], p["B"], p["h"], p["s"], p["G"], p["k"], X=p["X"], ws=ws)

    res = {}
    res["plain_fp64_solves_per_s"] = timed(plain)
    ms.check_status(ws)
    X_plain = [p["X"].clone() for p in p64]
    r64 = ms.BatchRunner(p64)
    res["batched_fp64_solves_per_s"] = timed(lambda: r64.launch())
    assert r64.status()[0] == ms.MS_OK
    X_b64 = [p["X"].clone() for p in p64]
    X_m = {}
    for rs in sorted({0, 1, refine}):
        rm = ms.BatchRunner(pbf, refine_steps=rs)
        res["batched_mixed_refine%d_solves_per_s" % rs] = timed(lambda: rm.launch())
        assert rm.status()[0] == ms.MS_OK
        X_m[rs] = [p["X"].clone() for p in pbf]
        del rm
    # early stop: up to 3 steps, a problem stops once its correction is at
    # most 2^-30 of its X
    rm = ms.BatchRunner(pbf, refine_steps=3, refine_tol_log2=30)
    res["batched_mixed_refine3_stop30_solves_per_s"] = timed(lambda: rm.launch())
    assert rm.status()[0] == ms.MS_OK
    X_stop = [p["X"].clone() for p in pbf]
    del rm
    res["batched_mixed_norefine_solves_per_s"] = res["batched_mixed_refine0_solves_per_s"]
    res["batched_mixed_solves_per_s"] = res["batched_mixed_refine%d_solves_per_s" % refine]

    def rhos(Xs):
        vals = []
        for p, X, xo in zip(p64, Xs, x_opt):
            num = torch.linalg.norm(p["B"] - p["A"] @ X)
            den = torch.linalg.norm(p["B"] - p["A"] @ xo)
            vals.append(float(num / den))
        return np.array(vals)

    def summ(v):
        return {"max": float(v.max()), "median": float(np.median(v)),
                "fraction_le_2": float(np.mean(v <= 2.0))}

    x_opt = []
    for p in p64:
        Q, R = torch.linalg.qr(p["A"], mode="reduced")
        x_opt.append(torch.linalg.solve_triangular(R, Q.t() @ p["B"], upper=True))
        del Q, R
    rho64 = rhos(X_b64)
    rho_m = {rs: rhos(X) for rs, X in X_m.items()}
    res["rho_vs_fp64_qr_optimum"] = dict(
        {"plain_fp64": summ(rhos(X_plain)), "batched_fp64": summ(rho64),
         "batched_mixed_refine3_stop30": summ(rhos(X_stop))},
        **{"batched_mixed_refine%d" % rs: summ(v) for rs, v in rho_m.items()})
    # the headline ratio: batched mixed precision against batched plain FP64
    # (the same batching, so the ratio isolates the precision), for the fewest
    # refinement steps at which every problem's residual ratio is within 2,
    # or within the FP64 sketch-and-solve's own ratio where that exceeds 2
    # (the sketch's distortion, which no precision removes), to 1e-3
    allow = np.maximum(2.0, rho64) * (1.0 + 1e-3)
    ok = [rs for rs in sorted(rho_m) if np.all(rho_m[rs] <= allow)]
    ok2 = [rs for rs in sorted(rho_m) if np.all(rho_m[rs] <= 2.0)]
    best = ok[0] if ok else refine
    res["mixed_refine_steps_for_rho_le_max_2_fp64"] = best if ok else None
    res["mixed_refine_steps_for_rho_le_2"] = ok2[0] if ok2 else None
    res["fp64_problems_with_rho_above_2"] = int(np.sum(rho64 > 2.0))
    res["ratio_batched_mixed_over_batched_fp64"] = (
        res["batched_mixed_refine%d_solves_per_s" % best] / res["batched_fp64_solves_per_s"])
    res["speedup_batched_mixed_over_plain_fp64"] = (
        res["batched_mixed_refine%d_solves_per_s" % best] / res["plain_fp64_solves_per_s"])
    res.update({"problems": count, "refine_steps": refine, "workload": SERVE_WORKLOAD,
                "g_dtype_mixed": "bf16", "reps": reps})
    return res


def rcq_leg(ms, torch, np, A, B, h, s, G, k, mode, X_ss, reps, A_host=None, B_host=None,
            h_host=None, s_host=None, G_host=None, cpu=True):
    """rand_cholQR least squares (Alg. 5) on the headline problem: solves/s
    and how close it and the sketch-and-solve x come to the least-squares
    optimum, measured by ||A^T r|| / (||A||_F ||r||) (zero at the optimum;
    the sketch-and-solve x carries the sketch's distortion).  With cpu, the
    oracle's rand_cholQR solve of the same arrays is timed once beside it."""
    X, R, ws = ms.rand_cholqr_lstsq(A, B, h, s, G, k, mode=mode)
    for _ in range(3):
        ms.rand_cholqr_lstsq(A, B, h, s, G, k, mode=mode, X=X, ws=ws)
    ms.check_status(ws)
    evs = [event_pair(torch) for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        ms.rand_cholqr_lstsq(A, B, h, s, G, k, mode=mode, X=X, ws=ws)
        e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms.check_status(ws)
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    anorm = float(torch.linalg.norm(A))

    def optimality(Xv):
        r = B - A @ Xv
        return float(torch.linalg.norm(A.t() @ r) / (anorm * torch.linalg.norm(r)))

    # the normal equations (Sec. 6.3's comparator) on the same problem
    Xn, _, nws = ms.normal_equations_lstsq(A, B)
    for _ in range(3):
        ms.normal_equations_lstsq(A, B, X=Xn, ws=nws)
    ms.check_status(nws)
    nevs = [event_pair(torch) for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in nevs:
        e0.record()
        ms.normal_equations_lstsq(A, B, X=Xn, ws=nws)
        e1.record()
    torch.cuda.synchronize()
    nwall = time.perf_counter() - t0
    ms.check_status(nws)
    nlat = np.array([a.elapsed_time(b) for a, b in nevs])
    out = {"solves_per_s": reps / wall, "ms_per_solve": 1e3 * wall / reps,
           "latency_ms": {"p50": float(np.percentile(lat, 50)),
                          "p99": float(np.percentile(lat, 99))},
           "normal_equations": {"solves_per_s": reps / nwall, "ms_per_solve": 1e3 * nwall / reps,
                                "latency_ms_p50": float(np.percentile(nlat, 50)),
                                "optimality": optimality(Xn),
                                "rel_diff_vs_rand_cholqr":
                                    float(torch.linalg.norm(Xn - X) / torch.linalg.norm(X))},
           "optimality_note": "||A^T r|| / (||A||_F ||r||); with b = A x* + 1e-6 N(0,1) the "
                              "rounding of r alone gives about u ||b|| / ||r|| = 1e-9",
           "residual_ratio_sketch_and_solve": float(torch.linalg.norm(B - A @ X_ss)
                                                    / torch.linalg.norm(B - A @ X)),
           "optimality_rand_cholqr": optimality(X),
           "optimality_sketch_and_solve": optimality(X_ss),
           "gram_pass_flops": 2 * A.shape[0] * A.shape[1] * (A.shape[1] + 1)
                              + 2 * A.shape[0] * A.shape[1] * B.shape[1],
           "gram_pass_bytes": A.shape[0] * (A.shape[1] + B.shape[1]) * A.element_size()}
    if cpu and A_host is not None:
        import oracle
        c0 = time.perf_counter()
        Xo, _, _ = oracle.rand_cholqr_lstsq(A_host, B_host, h_host, s_host, G_host, k)
        tc = time.perf_counter() - c0
        Xh = X.cpu().numpy()
        out["cpu_oracle"] = {"value": 1.0 / tc, "unit": "solves/s", "cores": 1, "kind": "oracle",
                             "sample": "1 full rand_cholQR solve of the same problem (%.1f s)"
                                       % tc,
                             "rel_err_gpu_vs_oracle":
                                 float(np.linalg.norm(Xh - Xo) / np.linalg.norm(Xo))}
    return out


def hashed_leg(ms, torch, seed, dev, reps=20):
    """The hash-generated CountSketch (Sec. 8's future-work variant) on the
    narrow workload where stored (h, s) matter most: A 16,777,216 x 8 FP32,
    k = 2 n^2 = 128.  Times the LDS CountSketch with stored packed codes
    (4 bytes per row), with stored h and s (5 bytes per row, checked in the
    kernel) and with generated ones (0 bytes per row)."""
    d, n, k = 1 << 24, 8, 128
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    A = torch.randn((n, d), generator=gen, device=dev, dtype=torch.float32).t()
    h, s = ms.hash_sketch(d, k, seed)
    code, _ = ms.pack_sketch(h, s, k)
    Y = ms.empty_colmajor(k, n, torch.float32, dev)
    cws = ms.workspace(ms.workspace_size("countsketch", d=d, n=n, k=k, a_dtype=ms.MS_F32), dev)
    hws = ms.workspace(ms.workspace_size("countsketch_hashed", d=d, n=n, k=k, a_dtype=ms.MS_F32),
                       dev)

    def timed(fn):
        for _ in range(3):
            fn()
        a, b = event_pair(torch)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e3  # us

    t_code = timed(lambda: ms.countsketch_accumulate(A, code, k, Y, mode="lds", ws=cws))
    t_hs = timed(lambda: ms.countsketch_apply(A, h, s, k, Y=Y, mode="lds", ws=cws))
    t_hash = timed(lambda: ms.countsketch_hashed(A, k, seed, Y=Y, ws=hws))
    ms.check_status(hws)
    base = d * n * 4 + k * n * 4
    out = {"workload": "countsketch_f32_16777216x8_k128", "bytes_A_and_Y": base}
    for name, t, extra in (("stored_packed_codes", t_code, 4 * d),
                           ("stored_h_s", t_hs, 5 * d),
                           ("hash_generated", t_hash, 0)):
        out[name] = {"avg_us": t, "algorithmic_bytes": base + extra,
                     "GBps": (base + extra) / (t * 1e-6) / 1e9,
                     "pct_hbm_peak": 100.0 * (base + extra) / (t * 1e-6) / 1e9 / HBM_PEAK_GBPS}
    out["speedup_vs_packed_codes"] = t_code / t_hash
    return out


def srht_leg(ms, torch, np, A, B, h, s, G, k, mode, X_ss, seed, reps=10):
    """The SRHT (Sec. 5) of the headline A (k = 2n rows, the paper's choice)
    against the CountSketch of the same A, and sketch-and-solve with the
    Count + SRHT multisketch against the Count + Gaussian one (same C,
    k2 = 2n), on the same problem."""
    d, n = A.shape
    k2 = G.shape[0]
    gen = torch.Generator(device=A.device)
    gen.manual_seed(seed)
    dsign = (torch.randint(0, 2, (d,), generator=gen, device=A.device, dtype=torch.int8) * 2 - 1)
    r = torch.randint(0, d, (2 * n,), generator=gen, device=A.device, dtype=torch.int32)
    Y, sws = ms.srht_apply(A, dsign, r)

    def timed(fn, nrep=reps):
        for _ in range(3):
            fn()
        a, b = event_pair(torch)
        a.record()
        for _ in range(nrep):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / nrep * 1e3  # us

    t_srht = timed(lambda: ms.srht_apply(A, dsign, r, Y=Y, ws=sws))
    ms.check_status(sws)
    bytes_srht = d * n * 8 + d + 2 * n * 4 + 2 * n * n * 8
    k1 = k
    m1 = 1 << (k1 - 1).bit_length()
    ds2 = (torch.randint(0, 2, (k1,), generator=gen, device=A.device, dtype=torch.int8) * 2 - 1)
    r2 = torch.randint(0, m1, (k2,), generator=gen, device=A.device, dtype=torch.int32)
    Xs, cws = ms.count_srht_lstsq(A, B, h, s, k1, ds2, r2, mode=mode)
    t_cs = timed(lambda: ms.count_srht_lstsq(A, B, h, s, k1, ds2, r2, mode=mode, X=Xs, ws=cws))
    ms.check_status(cws)
    Xg, gws = ms.sketch_lstsq(A, B, h, s, G, k, mode=mode)
    t_cg = timed(lambda: ms.sketch_lstsq(A, B, h, s, G, k, mode=mode, X=Xg, ws=gws))
    Xo, _, ows = ms.rand_cholqr_lstsq(A, B, h, s, G, k)  # the optimum (its residual)
    ms.check_status(ows)
    ropt = float(torch.linalg.norm(B - A @ Xo))
    return {"srht_4194304x64_k128": {"avg_us": t_srht, "algorithmic_bytes": bytes_srht,
                                     "GBps": bytes_srht / (t_srht * 1e-6) / 1e9,
                                     "pct_hbm_peak": 100.0 * bytes_srht / (t_srht * 1e-6) / 1e9
                                     / HBM_PEAK_GBPS},
            "count_srht_lstsq": {"avg_us": t_cs, "solves_per_s": 1e6 / t_cs,
                                 "rho": float(torch.linalg.norm(B - A @ Xs)) / ropt},
            "count_gaussian_lstsq": {"avg_us": t_cg, "solves_per_s": 1e6 / t_cg,
                                     "rho": float(torch.linalg.norm(B - A @ Xg)) / ropt}}


def other_configs_leg(ms, torch, np, seed, dev, reps=10, only=None):
    """The FP32 and mixed-precision least-squares workloads: full solves
    (sketch_lstsq) and their CountSketch kernel alone, inputs generated on
    the device from the seed (A = Z D [Q], b = A x* + 1e-6 N(0,1))."""
    out = {}
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    cases = [
        ("fp32_ill_conditioned_16777216x128", 1 << 24, 128, 1, 32768, 256, 1e6, True, "f32", 0),
        ("mixed_bf16_refine3_8388608x256", 1 << 23, 256, 4, 131072, 512, 1e4, False, "bf16", 3),
    ]
    for name, d, n, nrhs, k, k2, kappa, rotate, gd, refine in cases:
        if only and not name.startswith(only):
            continue
        scales = torch.logspace(0.0, -math.log10(kappa), n, device=dev, dtype=torch.float64)
        M = torch.diag(scales)
        if rotate:
            q, _ = torch.linalg.qr(torch.randn((n, n), generator=gen, device=dev,
                                               dtype=torch.float64))
            M = M @ q
        A = ms.empty_colmajor(d, n, torch.float32, dev)
        for r0 in range(0, d, 1 << 21):
            r1 = min(d, r0 + (1 << 21))
            Z = torch.randn((r1 - r0, n), generator=gen, device=dev, dtype=torch.float64)
            A[r0:r1].copy_(Z @ M)
        del Z
        xs = torch.randn((n, nrhs), generator=gen, device=dev, dtype=torch.float64)
        B = ms.empty_colmajor(d, nrhs, torch.float32, dev)
        for r0 in range(0, d, 1 << 21):
            r1 = min(d, r0 + (1 << 21))
            B[r0:r1].copy_(A[r0:r1].double() @ xs + 1e-6 * torch.randn(
                (r1 - r0, nrhs), generator=gen, device=dev, dtype=torch.float64))
        h = torch.randint(0, k, (d,), generator=gen, device=dev, dtype=torch.int32)
        s = (torch.randint(0, 2, (d,), generator=gen, device=dev, dtype=torch.int8) * 2 - 1)
        G = ms.empty_colmajor(k2, k, torch.bfloat16 if gd == "bf16" else torch.float32, dev)
        G.copy_(torch.randn((k, k2), generator=gen, device=dev, dtype=torch.float32).t()
                / math.sqrt(k2))
        X = ms.empty_colmajor(n, nrhs, torch.float64, dev)
        ws = ms.workspace(ms.workspace_size("lstsq", d=d, n=n, nrhs=nrhs, k=k, k2=k2,
                                            a_dtype=ms.MS_F32,
                                            g_dtype=ms.MS_BF16 if gd == "bf16" else ms.MS_F32,
                                            refine_steps=refine), dev)
        torch.cuda.synchronize()

        def solve():
            ms.sketch_lstsq(A, B, h, s, G, k, refine_steps=refine, X=X, ws=ws)

        solve()
        ms.check_status(ws)
        e0, e1 = event_pair(torch)
        e0.record()
        for _ in range(reps):
            solve()
        e1.record()
        torch.cuda.synchronize()
        ms.check_status(ws)
        solve_ms = e0.elapsed_time(e1) / reps
        # the CountSketch of [A | B] alone (the kernel the solve runs first)
        AB = ms.empty_colmajor(d, n + nrhs, torch.float32, dev)
        AB[:, :n].copy_(A)
        AB[:, n:].copy_(B)
        del A, B
        code, _ = ms.pack_sketch(h, s, k)
        Y = ms.empty_colmajor(k, n + nrhs, torch.float32, dev)
        # a workspace with room for the per-die partial sums, as in the solve
        cws = ms.workspace(ms.workspace_size("countsketch", d=d, n=n + nrhs, k=k,
                                             a_dtype=ms.MS_F32), dev)
        ms.countsketch_accumulate(AB, code, k, Y, mode="lds", ws=cws)
        e0.record()
        for _ in range(reps):
            ms.countsketch_accumulate(AB, code, k, Y, mode="lds", ws=cws)
        e1.record()
        torch.cuda.synchronize()
        ms.check_status(cws)
        cs_ms = e0.elapsed_time(e1) / reps
        cs_bytes = d * (n + nrhs) * 4 + d * 4 + k * (n + nrhs) * 4
        out[name] = {"d": d, "n": n, "nrhs": nrhs, "k": k, "k2": k2, "g_dtype": gd,
                     "refine_steps": refine, "ms_per_solve": solve_ms,
                     "solves_per_s": 1e3 / solve_ms,
                     "countsketch": {"avg_us": cs_ms * 1e3,
                                     "GBps": cs_bytes / (cs_ms * 1e-3) / 1e9,
                                     "frac_hbm_peak": cs_bytes / (cs_ms * 1e-3) / 1e9
                                     / HBM_PEAK_GBPS, "bytes_per_launch": cs_bytes}}
        del AB, Y, G, h, s, ws, X, code
        torch.cuda.empty_cache()
    return out


def c1_leg(ms, torch, seed, dev, reps=64):
    """The plain CountSketch workload, A 65,536 x 32 FP64 (16.8 MB), k = 2048:
    warm (the same A every call, resident in the 256 MB Infinity Cache) and
    cold (64 distinct copies of A, 1.07 GB, taken in turn, so each call's A
    comes from HBM).  Bytes per call: A, the 4-byte packed bucket/sign word
    per row, Y written once."""
    d, n, k = 65536, 32, 2048
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    copies = [torch.randn((n, d), generator=gen, device=dev, dtype=torch.float64).t()
              for _ in range(64)]
    h = torch.randint(0, k, (d,), generator=gen, device=dev, dtype=torch.int32)
    s = (torch.randint(0, 2, (d,), generator=gen, device=dev, dtype=torch.int8) * 2 - 1)
    code, _ = ms.pack_sketch(h, s, k)
    Y = ms.empty_colmajor(k, n, torch.float64, dev)
    cws = ms.workspace(ms.workspace_size("countsketch", d=d, n=n, k=k), dev)
    nbytes = d * n * 8 + d * 4 + k * n * 8

    def timed(pick):
        for i in range(8):
            ms.countsketch_accumulate(pick(i), code, k, Y, mode="lds", ws=cws)
        e0, e1 = event_pair(torch)
        e0.record()
        for i in range(reps):
            ms.countsketch_accumulate(pick(i), code, k, Y, mode="lds", ws=cws)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    def graphed(pick):
        # the same calls captured in one HIP graph and replayed: the kernels'
        # own time, without the host's per-call submission
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for i in range(reps):
                ms.countsketch_accumulate(pick(i), code, k, Y, mode="lds", ws=cws, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(reps):
                ms.countsketch_accumulate(pick(i), code, k, Y, mode="lds", ws=cws,
                                          stream=torch.cuda.current_stream())
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = event_pair(torch)
        e0.record()
        for _ in range(4):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        del g
        return e0.elapsed_time(e1) / (4 * reps) * 1e-3

    t_warm = timed(lambda i: copies[0])
    t_cold = timed(lambda i: copies[i % 64])
    g_warm = graphed(lambda i: copies[0])
    g_cold = graphed(lambda i: copies[i % 64])
    ms.check_status(cws)
    out = {"workload": "countsketch_65536x32_f64_k2048", "bytes_per_call": nbytes,
           "warm": {"avg_us": t_warm * 1e6, "GBps": nbytes / t_warm / 1e9,
                    "pct_hbm_peak": 100.0 * nbytes / t_warm / 1e9 / HBM_PEAK_GBPS},
           "cold_rotating_1GiB": {"avg_us": t_cold * 1e6, "GBps": nbytes / t_cold / 1e9,
                                  "pct_hbm_peak": 100.0 * nbytes / t_cold / 1e9 / HBM_PEAK_GBPS},
           "graph_replay": {
               "warm": {"avg_us": g_warm * 1e6, "GBps": nbytes / g_warm / 1e9,
                        "pct_hbm_peak": 100.0 * nbytes / g_warm / 1e9 / HBM_PEAK_GBPS},
               "cold_rotating_1GiB": {"avg_us": g_cold * 1e6, "GBps": nbytes / g_cold / 1e9,
                                      "pct_hbm_peak": 100.0 * nbytes / g_cold / 1e9 /
                                      HBM_PEAK_GBPS}},
           "note": "one call moves 17.6 MB; called from Python each call waits for its host "
                   "submission, so the graph replay (64 calls captured once) gives the "
                   "kernels' own rate"}
    del copies, Y, cws
    return out


def host_info():
    """nproc, the cores this process may run on, CPU model and RAM of the host."""
    info = {"nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def paper_comparison_leg(ms, torch, np, seed, dev, reps=5):
    """Sec. 6.3 / Sec. 8's headline comparison on this GPU: multisketch
    sketch-and-solve against the normal equations at d = 2^22, n = 256,
    kappa(A) = 1e2, FP64, with the paper's "easy" right-hand side
    b = A e + N(0, 0.01) (k = 2 n^2 = 131,072, k2 = 2 n = 512).  Inputs are
    generated on the device from the seed; both solvers go through the C ABI
    and are timed with events.  x_opt for the residual ratio comes from a
    library QR least-squares solve in FP64 on the device (measurement only)."""
    d, n, kappa = 1 << 22, 256, 1e2
    k, k2 = 2 * n * n, 2 * n
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    scales = torch.logspace(0.0, -math.log10(kappa), n, device=dev, dtype=torch.float64)
    q, _ = torch.linalg.qr(torch.randn((n, n), generator=gen, device=dev, dtype=torch.float64))
    M = torch.diag(scales) @ q
    A = ms.empty_colmajor(d, n, torch.float64, dev)
    for r0 in range(0, d, 1 << 20):
        r1 = min(d, r0 + (1 << 20))
        A[r0:r1].copy_(torch.randn((r1 - r0, n), generator=gen, device=dev,
                                   dtype=torch.float64) @ M)
    b = ms.empty_colmajor(d, 1, torch.float64, dev)
    b.copy_(A.sum(dim=1, keepdim=True) + 0.1 * torch.randn((d, 1), generator=gen, device=dev,
                                                           dtype=torch.float64))
    h = torch.randint(0, k, (d,), generator=gen, device=dev, dtype=torch.int32)
    s = (torch.randint(0, 2, (d,), generator=gen, device=dev, dtype=torch.int8) * 2 - 1)
    G = ms.empty_colmajor(k2, k, torch.float64, dev)
    G.copy_(torch.randn((k, k2), generator=gen, device=dev, dtype=torch.float64).t()
            / math.sqrt(k2))
    Xs = ms.empty_colmajor(n, 1, torch.float64, dev)
    wss = ms.workspace(ms.workspace_size("lstsq", d=d, n=n, nrhs=1, k=k, k2=k2), dev)
    Xn, _, wne = ms.normal_equations_lstsq(A, b)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        e0, e1 = event_pair(torch)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_ss = timed(lambda: ms.sketch_lstsq(A, b, h, s, G, k, X=Xs, ws=wss))
    ms.check_status(wss)
    t_ne = timed(lambda: ms.normal_equations_lstsq(A, b, X=Xn, ws=wne))
    ms.check_status(wne)
    xo = torch.linalg.lstsq(A, b).solution
    bn = b.norm().item()

    def res(x):
        return (b - A @ x).norm().item()

    r_opt = res(xo)
    out = {"workload": "d=4,194,304 n=256 kappa(A)=1e2 FP64, b = A e + N(0, 0.01); "
                       "multisketch k=131,072 k2=512",
           "sketch_and_solve": {"ms_per_solve": t_ss, "solves_per_s": 1e3 / t_ss,
                                "relative_residual": res(Xs) / bn, "rho": res(Xs) / r_opt},
           "normal_equations": {"ms_per_solve": t_ne, "solves_per_s": 1e3 / t_ne,
                                "relative_residual": res(Xn) / bn, "rho": res(Xn) / r_opt},
           "time_ratio_normal_equations_over_sketch_and_solve": t_ne / t_ss,
           "paper": "multisketch sketch-and-solve 'up to 77% faster' than the normal equations "
                    "at d = 2^22, n = 256 on an H100 (abstract, Sec. 8); quoted, not converted"}
    del A, b, h, s, G, wss, wne, xo
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU row-block reduction is a design note, not a code path)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2508_14209_amd as ms
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.only == "copy":
        nbytes = 1 << 30
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).normal_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"only": "copy", "bytes_read_per_launch": nbytes,
                          "bytes_written_per_launch": nbytes, "launches": args.steps}))
        return
    if args.only == "srht":
        # the SRHT of A 4,194,304 x 64 FP64 (k = 128 sampled rows) alone
        d_, n_, k_ = 4194304, 64, 128
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        Ax = torch.randn((n_, d_), generator=gen, device=dev, dtype=torch.float64).t()
        dx = (torch.randint(0, 2, (d_,), generator=gen, device=dev, dtype=torch.int8) * 2 - 1)
        rx = torch.randint(0, d_, (k_,), generator=gen, device=dev, dtype=torch.int32)
        Yx, sws = ms.srht_apply(Ax, dx, rx)
        for _ in range(args.steps):
            ms.srht_apply(Ax, dx, rx, Y=Yx, ws=sws)
        ms.check_status(sws)
        print(json.dumps({"only": args.only, "kernel": "k_srht_block", "launches": args.steps + 1,
                          "bytes_per_launch": d_ * n_ * 8 + d_ + k_ * 4 + k_ * n_ * 8}))
        return
    if args.only == "countsketch_hashed":
        # the hash-generated CountSketch of A 16,777,216 x 8 FP32 (k = 128) alone
        d_, n_, k_ = 1 << 24, 8, 128
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        Ax = torch.randn((n_, d_), generator=gen, device=dev, dtype=torch.float32).t()
        Yx, hws = ms.countsketch_hashed(Ax, k_, args.seed)
        for _ in range(args.steps):
            ms.countsketch_hashed(Ax, k_, args.seed, Y=Yx, ws=hws)
        ms.check_status(hws)
        print(json.dumps({"only": args.only, "kernel": "k_cs_lds_xcd (hashed)",
                          "launches": args.steps + 1, "bytes_per_launch": d_ * n_ * 4 + k_ * n_ * 4}))
        return
    if args.only == "paper_comparison":
        # sketch-and-solve against the normal equations at 4,194,304 x 256
        print(json.dumps(paper_comparison_leg(ms, torch, np, args.seed + 5, dev, reps=2)))
        return
    if args.only in ("solve_fp32", "solve_mixed"):
        # one of the FP32 / mixed-precision solves alone (3 timed solves)
        res = other_configs_leg(ms, torch, np, args.seed + 2, dev, reps=3,
                                only="fp32" if args.only == "solve_fp32" else "mixed")
        print(json.dumps(res))
        return
    if args.only in ("batched_mixed", "batched_fp64"):
        # the batched mixed-precision (or plain FP64) solve of the comparison batch, alone
        p64, pbf = compare_problems(ms, torch, args.compare_problems, args.seed + 1, dev)
        if args.only == "batched_fp64":
            r = ms.BatchRunner(p64)
            for _ in range(args.steps):
                r.launch()
            torch.cuda.synchronize()
            print(json.dumps({"only": args.only, "problems": len(p64),
                              "status": r.status()[0], "launches": args.steps}))
            return
        r = ms.BatchRunner(pbf, refine_steps=args.refine)
        for _ in range(args.steps):
            r.launch()
        torch.cuda.synchronize()
        print(json.dumps({"only": args.only, "problems": len(pbf), "refine_steps": args.refine,
                          "status": r.status()[0], "launches": args.steps}))
        return
    if args.only in ("countsketch_f32_k32768", "countsketch_f32_k131072"):
        # the FP32 workloads' CountSketch of [A | B] alone (device-generated
        # N(0,1) data of the workload's shape; the kernel does not depend on
        # the values)
        big = args.only.endswith("131072")
        d_, nc_, k_ = ((1 << 23), 260, 131072) if big else ((1 << 24), 129, 32768)
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        ABx = ms.empty_colmajor(d_, nc_, torch.float32, dev)
        for c in range(nc_):
            ABx[:, c].normal_(generator=gen)
        hx = torch.randint(0, k_, (d_,), generator=gen, device=dev, dtype=torch.int32)
        sx = (torch.randint(0, 2, (d_,), generator=gen, device=dev, dtype=torch.int8) * 2 - 1)
        code, _ = ms.pack_sketch(hx, sx, k_)
        Yx = ms.empty_colmajor(k_, nc_, torch.float32, dev)
        cws = ms.workspace(ms.workspace_size("countsketch", d=d_, n=nc_, k=k_,
                                             a_dtype=ms.MS_F32), dev)
        Yx.zero_()
        torch.cuda.synchronize()
        for _ in range(args.steps):
            ms.countsketch_accumulate(ABx, code, k_, Yx, mode="lds", ws=cws)
        ms.check_status(cws)
        print(json.dumps({"only": args.only, "kernel": "k_cs_tiled", "launches": args.steps,
                          "bytes_per_launch": d_ * nc_ * 4 + d_ * 4 + k_ * nc_ * 4}))
        return
    if args.only == "countsketch_sorted":
        # the deterministic CountSketch of [A | b] (4,194,304 x 65 FP64, k =
        # 8192): per-block sorted keys, then the block-ordered fold (each
        # bucket summed in ascending row order); and the bucket plan alone
        # (ms_bucket_plan)
        d_, nc_, k_ = 4194304, 65, 8192
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        ABx = torch.randn((nc_, d_), generator=gen, device=dev, dtype=torch.float64).t()
        hx = torch.randint(0, k_, (d_,), generator=gen, device=dev, dtype=torch.int32)
        sx = (torch.randint(0, 2, (d_,), generator=gen, device=dev, dtype=torch.int8) * 2 - 1)
        Yx, sws = ms.countsketch_apply(ABx, hx, sx, k_, mode="sorted")
        cnt, off, perm, pws = ms.bucket_plan(hx, k_)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            ms.countsketch_apply(ABx, hx, sx, k_, mode="sorted", Y=Yx, ws=sws)
            ms.bucket_plan(hx, k_, ws=pws)
        ms.check_status(sws)
        ms.check_status(pws)
        print(json.dumps({"only": args.only, "kernels": "k_bf_keys_count (k <= 16384; k_bf_keys above) + k_bf_fold (sketch), k_pb_* (plan)",
                          "launches": args.steps + 1,
                          "bytes_per_launch": {"fold": d_ * nc_ * 8 + d_ * 4 + k_ * nc_ * 8,
                                               "plan": d_ * 4 + d_ * 4 + 2 * k_ * 4}}))
        return
    if args.only in ("gaussian_f64", "gaussian_bf16"):
        # Gaussian stage alone on device-generated inputs of the workload's shape
        bf = args.only == "gaussian_bf16"
        k2_, k_, nc_ = (512, 131072, 260) if bf else (128, 8192, 65)
        gen = torch.Generator(device=dev)
        gen.manual_seed(args.seed)
        G32 = torch.randn((k_, k2_), generator=gen, device=dev, dtype=torch.float64).t()
        G32.mul_(1.0 / math.sqrt(k2_))
        Gx = ms.empty_colmajor(k2_, k_, torch.bfloat16 if bf else torch.float64, dev)
        Gx.copy_(G32)
        Yx = ms.empty_colmajor(k_, nc_, torch.float32 if bf else torch.float64, dev)
        Yx.copy_(torch.randn((nc_, k_), generator=gen, device=dev, dtype=torch.float64).t())
        del G32
        Zx, gws_ = ms.gaussian_apply(Gx, Yx)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            ms.gaussian_apply(Gx, Yx, Z=Zx, ws=gws_)
        torch.cuda.synchronize()
        print(json.dumps({"only": args.only, "k2": k2_, "k": k_, "ncols": nc_,
                          "flops_per_call": 2 * k2_ * k_ * nc_, "launches": args.steps}))
        return
    d, n, nrhs, k, k2 = 4194304, 64, 1, 8192, 128
    nc = n + nrhs
    seed = args.seed

    # ---- inputs (host, seeded), then resident in HBM: [A | b] in one buffer
    A = synth.normal_matrix(d, n, seed=seed)
    B, _ = synth.lstsq_rhs(A, nrhs, seed=seed)
    h = synth.bucket_map(d, k, seed=seed)
    s = synth.signs(d, seed=seed)
    G = synth.gaussian_sketch(k2, k, seed=seed)
    AB = ms.empty_colmajor(d, nc, torch.float64, dev)
    AB[:, :n].copy_(torch.from_numpy(np.ascontiguousarray(A.T)).t())
    AB[:, n:].copy_(torch.from_numpy(np.ascontiguousarray(B.T)).t())
    Ad, Bd = AB[:, :n], AB[:, n:]
    Gd = ms.empty_colmajor(k2, k, torch.float64, dev)
    Gd.copy_(torch.from_numpy(np.ascontiguousarray(G.T)).t())
    hd = torch.from_numpy(h).to(dev)
    sd = torch.from_numpy(s).to(dev)
    X = ms.empty_colmajor(n, nrhs, torch.float64, dev)
    ws = ms.workspace(ms.workspace_size("lstsq", d=d, n=n, nrhs=nrhs, k=k, k2=k2,
                                        mode=args.mode), dev)
    torch.cuda.synchronize()
    if args.only == "normal_equations":
        # the normal equations of the headline problem alone
        Xn, _, nws = ms.normal_equations_lstsq(Ad, Bd)
        for _ in range(args.steps):
            ms.normal_equations_lstsq(Ad, Bd, X=Xn, ws=nws)
        ms.check_status(nws)
        print(json.dumps({"only": args.only, "kernel": "k_rcq_gram (plain)",
                          "launches": args.steps + 1,
                          "flops_per_launch": d * n * (n + 1) + 2 * d * n * nrhs,
                          "bytes_per_launch": d * nc * 8}))
        return
    if args.only == "rand_cholqr":
        # rand_cholQR least squares of the headline problem alone
        Xr, _, rws = ms.rand_cholqr_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode)
        for _ in range(args.steps):
            ms.rand_cholqr_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode, X=Xr, ws=rws)
        ms.check_status(rws)
        print(json.dumps({"only": args.only, "kernel": "k_rcq_gram", "launches": args.steps + 1,
                          "flops_per_launch": 2 * d * n * (n + 1) + 2 * d * n * nrhs,
                          "bytes_per_launch": d * nc * 8}))
        return
    if args.only == "countsketch":
        # the step's CountSketch kernel alone: codes packed once, then
        # args.steps launches of the LDS kernel over [A | b]
        code, _ = ms.pack_sketch(hd, sd, k)
        Y = ms.empty_colmajor(k, nc, torch.float64, dev)
        cws = ms.workspace(256, dev)
        Y.zero_()
        torch.cuda.synchronize()
        for _ in range(args.steps):
            ms.countsketch_accumulate(AB, code, k, Y, mode="lds", ws=cws)
        ms.check_status(cws)
        print(json.dumps({"only": "countsketch", "kernel": "k_cs_lds_xcd", "launches": args.steps,
                          "bytes_per_launch": d * nc * 8 + d * 4 + k * nc * 8}))
        return

    # ---- the step: one sketch-and-solve, W warm-up + K timed
    for _ in range(args.warmup):
        ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode, X=X, ws=ws)
    ms.check_status(ws)
    evs = [event_pair(torch) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode, X=X, ws=ws)
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms.check_status(ws)
    elapsed = t1 - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])  # ms, GPU time of each solve
    Xh = X.cpu().numpy()

    # ---- the same solve with two in flight (two streams, two workspaces):
    # independent requests of this size overlap one solve's QR and Gaussian
    # stage (a few compute units) with the other's CountSketch; reported
    # beside the one-at-a-time value, which stays the headline
    X2 = ms.empty_colmajor(n, nrhs, torch.float64, dev)
    _, ws2 = ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode, X=X2)
    pair = [(X, ws, torch.cuda.Stream()), (X2, ws2, torch.cuda.Stream())]
    torch.cuda.synchronize()
    for i in range(4):
        Xi, wsi, sti = pair[i % 2]
        ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode, X=Xi, ws=wsi, stream=sti)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for i in range(args.steps):
        Xi, wsi, sti = pair[i % 2]
        ms.sketch_lstsq(Ad, Bd, hd, sd, Gd, k, mode=args.mode, X=Xi, ws=wsi, stream=sti)
    torch.cuda.synchronize()
    two_wall = time.perf_counter() - tp0
    ms.check_status(ws2)
    two_in_flight = {"solves_per_s": args.steps / two_wall,
                     "ms_per_solve": 1e3 * two_wall / args.steps,
                     "max_abs_diff_vs_one_at_a_time": float((X2 - X).abs().max())}
    del ws2

    # ---- dominant kernel: LDS-binned CountSketch of [A | b], timed alone
    code, _ = ms.pack_sketch(hd, sd, k)
    Y = ms.empty_colmajor(k, nc, torch.float64, dev)
    Y.zero_()
    cws = ms.workspace(256, dev)
    reps = max(10, args.steps)

    def time_calls(fn, n_calls):
        for _ in range(3):
            fn()
        a, b = event_pair(torch)
        a.record()
        for _ in range(n_calls):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n_calls  # ms per call

    cs_ms = time_calls(lambda: ms.countsketch_accumulate(AB, code, k, Y, mode="lds", ws=cws), reps)
    ms.check_status(cws)
    # algorithmic bytes per launch: [A | b] read once, one 4-byte packed
    # bucket/sign word per row, the k x 65 sketch written once
    cs_bytes = d * nc * 8 + d * 4 + k * nc * 8
    cs_gbps = cs_bytes / (cs_ms * 1e-3) / 1e9
    at_ms = time_calls(lambda: ms.countsketch_accumulate(AB, code, k, Y, mode="atomic", ws=cws),
                       max(5, reps // 10))
    Ys = ms.empty_colmajor(k, nc, torch.float64, dev)
    sws = ms.workspace(ms.workspace_size("countsketch", d=d, n=nc, k=k, mode="sorted"), dev)
    so_ms = time_calls(lambda: ms.countsketch_apply(AB, hd, sd, k, Y=Ys, mode="sorted", ws=sws),
                       max(5, reps // 10))
    ms.check_status(sws)
    # Gaussian stage alone (FP64 matrix cores), on the sketch
    Z = ms.empty_colmajor(k2, nc, torch.float64, dev)
    gws = ms.workspace(ms.workspace_size("gaussian", n=nc, k=k, k2=k2), dev)
    gs_ms = time_calls(lambda: ms.gaussian_apply(Gd, Y, Z=Z, ws=gws), reps)
    gs_flops = 2.0 * k2 * k * nc

    # ---- rand_cholQR least squares on the same problem (its own leg)
    rcq = srht = None
    try:
        if not args.extras:
            raise StopIteration
        rcq = rcq_leg(ms, torch, np, Ad, Bd, hd, sd, Gd, k, args.mode, X, max(10, args.steps // 5),
                      A, B, h, s, G, cpu=args.cpu_seconds > 0)
    except StopIteration:
        pass
    except Exception as e:  # reported in the line, not hidden
        rcq = {"error": repr(e)}

    # ---- SRHT and the Count + SRHT multisketch on the same problem
    try:
        if args.extras:
            srht = srht_leg(ms, torch, np, Ad, Bd, hd, sd, Gd, k, args.mode, X, seed + 3)
    except Exception as e:
        srht = {"error": repr(e)}

    # ---- CPU baseline: the oracle on this host, same arrays.  All cores: the
    # oracle's CountSketch with its columns split over the host threads
    # (bit-identical to the sequential fold), then its Gaussian stage and QR
    # solve; one core: the oracle's single-threaded sketch_lstsq.
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        oracle.build(force=False)
        hi = host_info()
        threads = max(1, min(16, hi["usable_cores"]))
        AB = np.asfortranarray(np.hstack([A, B]))

        def solve_all_cores():
            Y = oracle.countsketch(AB, h, s, k, threads=threads)
            Z = oracle.gemm(G, Y)
            return oracle.qr_solve(Z[:, :n], Z[:, n:])

        def run(fn, budget):
            n_done, t_cpu, Xo = 0, 0.0, None
            while n_done < 1 or (t_cpu < budget and n_done < 20):
                c0 = time.perf_counter()
                Xo = fn()
                t_cpu += time.perf_counter() - c0
                n_done += 1
            return n_done, t_cpu, Xo

        na, ta, Xa = run(solve_all_cores, 0.5 * args.cpu_seconds)
        n1, t1, X1 = run(lambda: oracle.sketch_lstsq(A, B, h, s, G, k)[0], 0.5 * args.cpu_seconds)
        cpu = {"value": na / ta, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": "%d full solves of the same 4,194,304 x 64 FP64 problem on %d host "
                         "threads (plain C oracle; CountSketch columns split over the threads, "
                         "bit-identical to the sequential fold; %.1f s)" % (na, threads, ta),
               "single_core": {"value": n1 / t1, "cores": 1,
                               "sample": "%d solves, single-threaded oracle, %.1f s" % (n1, t1)},
               "all_cores_equals_single_core": bool(np.array_equal(Xa, X1)),
               "host": hi,
               "rel_err_gpu_vs_oracle": float(np.linalg.norm(Xh - X1) / np.linalg.norm(X1))}

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "d": d, "n": n, "nrhs": nrhs, "k": k, "k2": k2,
                   "a": "iid N(0,1)", "b": "A x* + 1e-6 N(0,1)", "cs_mode": args.mode,
                   "seed": seed},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "two_in_flight": two_in_flight,
        "countsketch": {"kernel": "k_cs_lds_xcd", "avg_us": cs_ms * 1e3, "GBps": cs_gbps,
                        "pct_hbm_peak": 100.0 * cs_gbps / HBM_PEAK_GBPS,
                        "bytes_per_launch": cs_bytes,
                        "atomic_baseline_GBps": cs_bytes / (at_ms * 1e-3) / 1e9,
                        "sorted_deterministic_GBps": (cs_bytes + d) / (so_ms * 1e-3) / 1e9},
        "gaussian_stage": {"avg_us": gs_ms * 1e3, "TFLOPs": gs_flops / (gs_ms * 1e-3) / 1e12,
                           "pct_fp64_peak": 100.0 * gs_flops / (gs_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS},
        "roofline": {"bound": "hbm", "achieved": cs_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": cs_gbps / HBM_PEAK_GBPS, "traffic": measured_traffic()},
        "cpu_baseline": cpu,
        "rand_cholqr": rcq,
        "srht": srht,
    }
    # beyond the headline: the serving loop and the batched mixed-precision
    # solver against the plain FP64 one (each leg reports its own error)
    del AB, Gd, Y, Ys, Z, ws, sws, gws
    torch.cuda.empty_cache()
    if args.serve_requests > 0:
        try:
            out["serving"] = serving_leg(ms, torch, np, args.serve_requests, seed, args.refine,
                                         dev)
        except Exception as e:  # reported in the line, not hidden
            out["serving"] = {"error": repr(e)}
    if args.other_configs:
        try:
            out["other_configs"] = other_configs_leg(ms, torch, np, seed + 2, dev)
        except Exception as e:
            out["other_configs"] = {"error": repr(e)}
    try:
        if args.extras:
            out["paper_comparison"] = paper_comparison_leg(ms, torch, np, seed + 5, dev)
    except Exception as e:
        out["paper_comparison"] = {"error": repr(e)}
    try:
        out["countsketch_65536x32"] = c1_leg(ms, torch, seed + 6, dev)
    except Exception as e:
        out["countsketch_65536x32"] = {"error": repr(e)}
    try:
        if args.extras:
            out["hashed_countsketch"] = hashed_leg(ms, torch, seed, dev)
    except Exception as e:
        out["hashed_countsketch"] = {"error": repr(e)}
    if args.compare_problems > 0:
        try:
            out["batched_mixed_vs_plain_fp64"] = mixed_vs_fp64_leg(
                ms, torch, np, args.compare_problems, seed + 1, args.refine, dev)
        except Exception as e:
            out["batched_mixed_vs_plain_fp64"] = {"error": repr(e)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
