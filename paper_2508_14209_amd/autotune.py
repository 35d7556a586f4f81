"""Autotuner for the library's tile shapes, with an on-disk cache.

Two tuners:
  * ``tune_countsketch`` -- for a CountSketch shape (d, columns, k, dtype):
    schedule (persistent die-aware / one workgroup per chunk) x columns binned
    per workgroup.
  * ``tune_batch`` -- for a batch of problems: rows per CountSketch work item x
    K per Gaussian-stage work item.

Each candidate is timed with HIP events over a few launches on the caller's
inputs; a candidate whose result differs from the default's beyond the
association-order tolerance is discarded.  The fastest is stored in a JSON
cache keyed by the device name and a shape class (d rounded to a power of
two), and ``lookup_*`` returns cached choices without timing.

Cache file: $MSKETCH_TUNE_CACHE, else ~/.cache/msketch/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import threading

import torch

import paper_2508_14209_amd as ms

_lock = threading.Lock()


def cache_path() -> str:
    p = os.environ.get("MSKETCH_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "msketch", "tune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict):
    with _lock:
        data = _load()
        data[key] = value
        path = cache_path()
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def _device_name(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return "%s:%s:%d" % (p.name, getattr(p, "gcnArchName", "?"), p.multi_processor_count)


def _time(fn, reps: int) -> float:
    for _ in range(2):
        fn()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def cs_key(d: int, ncols: int, k: int, dtype, device) -> str:
    return "cs|%s|%s|d2^%d|c%d|k%d" % (_device_name(device), str(dtype).replace("torch.", ""),
                                      max(0, round(math.log2(max(1, d)))), ncols, k)


def lookup_countsketch(d: int, ncols: int, k: int, dtype, device="cuda"):
    """(tile_cols, schedule) from the cache, or None."""
    v = _load().get(cs_key(d, ncols, k, dtype, torch.device(device)))
    return (v["tile_cols"], v["schedule"]) if v else None


def tune_countsketch(A: torch.Tensor, h: torch.Tensor, s: torch.Tensor, k: int,
                     reps: int = 5, store: bool = True) -> dict:
    """Time the LDS CountSketch variants on (A, h, s) and cache the fastest."""
    d, ncols = A.shape
    code, _ = ms.pack_sketch(h, s, k)
    Y = ms.empty_colmajor(k, ncols, A.dtype, A.device)
    ws = ms.workspace(256, A.device)
    tol = 1e-12 if A.dtype == torch.float64 else 1e-5
    Y.zero_()
    ms.countsketch_accumulate(A, code, k, Y, ws=ws)
    ref = Y.double().clone()
    results = []
    for schedule in (0, 1):
        for cols in (1, 2, 4, 8):
            if cols > ncols:
                continue
            Y.zero_()
            try:
                ms.countsketch_accumulate(A, code, k, Y, ws=ws, tile_cols=cols, schedule=schedule)
                ms.check_status(ws)
            except ms.MsketchError:
                continue
            err = float((Y.double() - ref).norm() / max(ref.norm().item(), 1e-300))
            if err > tol:
                continue
            t = _time(lambda: ms.countsketch_accumulate(A, code, k, Y, ws=ws, tile_cols=cols,
                                                        schedule=schedule), reps)
            results.append({"tile_cols": cols, "schedule": schedule, "ms": t})
    best = min(results, key=lambda r: r["ms"])
    best = dict(best, candidates=len(results))
    if store:
        _store(cs_key(d, ncols, k, A.dtype, A.device), best)
    return best


def batch_key(problems, device) -> str:
    """Shape class of a batch: dtypes, largest n (rounded up to a power of
    two) and mean d (nearest power of two).  The count is not part of it, so
    batches of a serving stream with similar requests share one entry."""
    n = max(int(p["A"].shape[1]) for p in problems)
    d = sum(int(p["A"].shape[0]) for p in problems) // len(problems)
    return "batch|%s|%s|%s|d2^%d|n<=%d" % (
        _device_name(device), str(problems[0]["A"].dtype).replace("torch.", ""),
        str(problems[0]["G"].dtype).replace("torch.", ""),
        max(0, round(math.log2(max(1, d)))), 1 << max(0, math.ceil(math.log2(max(1, n)))))


def lookup_batch(problems, device="cuda"):
    """(rows_log2, kchunk_log2) cached for the batch's shape class, or None."""
    v = _load().get(batch_key(problems, torch.device(device)))
    return (v["rows_log2"], v["kchunk_log2"]) if v else None


def batch_params(problems, device="cuda"):
    """Tuning for BatchRunner: the cached choice, else (0, 0) (library
    defaults)."""
    return lookup_batch(problems, device) or (0, 0)


def tune_batch(problems, reps: int = 3, store: bool = True,
               rows=(13, 14, 15, 16, 17), kchunks=(8, 9, 10, 11)) -> dict:
    """Time batched solves of ``problems`` over rows-per-item x K-per-item."""
    results = []
    ref = None
    for rl in rows:
        for kl in kchunks:
            r = ms.BatchRunner(problems, rows_log2=rl, kchunk_log2=kl)
            r.launch()
            st, _ = r.status()
            if st != ms.MS_OK:
                continue
            X = torch.cat([p["X"].reshape(-1) for p in problems])
            if ref is None:
                ref = X.clone()
            else:
                err = float((X - ref).norm() / max(ref.norm().item(), 1e-300))
                if not err <= 1e-3:
                    continue
            t = _time(r.launch, reps)
            results.append({"rows_log2": rl, "kchunk_log2": kl, "ms": t})
    best = dict(min(results, key=lambda q: q["ms"]), candidates=len(results))
    if store:
        _store(batch_key(problems, problems[0]["A"].device), best)
    return best
