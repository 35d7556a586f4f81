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
  * the CPU oracle on the host, for the cpu_baseline entry.

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
    ap.add_argument("--only", default=None, choices=["countsketch", "copy"],
                    help="profiling runs: launch only the LDS CountSketch of [A | b] (--steps "
                         "times) or only a plain device copy of 1 GiB (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters); prints a short JSON line")
    return ap.parse_args()


def event_pair(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


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

    # ---- CPU baseline: the oracle on this host, same arrays
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        oracle.build(force=False)
        n_done, t_cpu = 0, 0.0
        while n_done < 1 or (t_cpu < args.cpu_seconds and n_done < 20):
            c0 = time.perf_counter()
            Xo, _, _ = oracle.sketch_lstsq(A, B, h, s, G, k)
            t_cpu += time.perf_counter() - c0
            n_done += 1
        cpu = {"value": n_done / t_cpu, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "%d full solves of the same 4,194,304 x 64 FP64 problem (single-threaded "
                         "plain C oracle, %.1f s)" % (n_done, t_cpu),
               "rel_err_gpu_vs_oracle": float(np.linalg.norm(Xh - Xo) / np.linalg.norm(Xo))}

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
        "countsketch": {"kernel": "k_cs_lds_xcd", "avg_us": cs_ms * 1e3, "GBps": cs_gbps,
                        "pct_hbm_peak": 100.0 * cs_gbps / HBM_PEAK_GBPS,
                        "bytes_per_launch": cs_bytes,
                        "atomic_baseline_GBps": cs_bytes / (at_ms * 1e-3) / 1e9,
                        "sorted_deterministic_GBps": (cs_bytes + d) / (so_ms * 1e-3) / 1e9},
        "gaussian_stage": {"avg_us": gs_ms * 1e3, "TFLOPs": gs_flops / (gs_ms * 1e-3) / 1e12,
                           "pct_fp64_peak": 100.0 * gs_flops / (gs_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS},
        "roofline": {"bound": "hbm", "achieved": cs_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": cs_gbps / HBM_PEAK_GBPS, "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
