"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds none of the sketching or solving arithmetic: it only draws
random data (matrices, bucket maps, signs, Gaussian sketch matrices, right-hand
sides) from a seed, so that both sides of every parity check see identical
inputs.  Random numbers the method consumes (h, s, G) are data: they are drawn
here and passed in.

Generator: NumPy PCG64 seeded through ``SeedSequence``.  Large matrices are
filled in fixed blocks of ``BLOCK_ROWS`` rows per column, each block from its
own child sequence keyed by (seed, stream, column, block), so the values do not
depend on how many threads fill them.

Workloads (shapes and distributions follow the paper's experiments, Sec. 6.2
and 6.3: tall-skinny random A, CountSketch dimension k = 2n^2 and Gaussian
dimension k2 = 2n, condition numbers set through a log-spaced diagonal).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BLOCK_ROWS = 1 << 20

# named streams, in a fixed order
STREAM = {"A": 0, "Q": 1, "xstar": 2, "noise": 3, "h": 4, "s": 5, "G": 6,
          "B": 7, "arrivals": 8, "req": 9}


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _gen(seed: int, *key: int) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=int(seed), spawn_key=tuple(int(x) for x in key))
    return np.random.Generator(np.random.PCG64(ss))


def normal_matrix(d: int, n: int, seed: int, stream: str = "A",
                  dtype=np.float64, scale: float = 1.0) -> np.ndarray:
    """d x n column-major matrix of i.i.d. N(0, scale^2) entries."""
    dtype = np.dtype(dtype)
    out = np.empty((d, n), dtype=dtype, order="F")
    sid = STREAM[stream]
    jobs = [(c, b) for c in range(n) for b in range((d + BLOCK_ROWS - 1) // BLOCK_ROWS)]

    def fill(job):
        c, b = job
        r0 = b * BLOCK_ROWS
        r1 = min(d, r0 + BLOCK_ROWS)
        g = _gen(seed, sid, c, b)
        col = out[r0:r1, c]
        g.standard_normal(out=col, dtype=dtype)
        if scale != 1.0:
            col *= dtype.type(scale)

    if len(jobs) > 1 and d * n > (1 << 18):
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, jobs))
    else:
        for j in jobs:
            fill(j)
    return out


def bucket_map(d: int, k: int, seed: int) -> np.ndarray:
    """h[i] i.i.d. uniform on {0, ..., k-1} (0-based form of Def. 3's r_j)."""
    g = _gen(seed, STREAM["h"])
    return g.integers(0, k, size=d, dtype=np.int32)


def signs(d: int, seed: int) -> np.ndarray:
    """s[i] i.i.d. Rademacher (+1 / -1), stored as int8 (Def. 3's sigma_j)."""
    g = _gen(seed, STREAM["s"])
    return (g.integers(0, 2, size=d, dtype=np.int8) * 2 - 1).astype(np.int8)


def to_bf16_values(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even) via FP32; returned as
    float32 holding BF16-representable values.  Used to define a BF16 input
    (the Gaussian matrix G of the mixed-precision path) once, for both sides."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    isnan = np.isnan(f)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    r = np.where(isnan, (u.astype(np.uint32) | 0x00400000) & 0xFFFF0000, r)
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(x))


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """The 16-bit BF16 patterns of float32 values that are BF16-representable."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def gaussian_sketch(k2: int, k: int, seed: int, dtype: str = "f64") -> np.ndarray:
    """G (k2 x k), entries N(0, 1/k2) (variance 1/k2, Sec. 1), column-major.

    dtype 'f64' -> float64; 'f32' -> float32 rounding of the same draw;
    'bf16' -> BF16 rounding (via FP32, ties to even) held in float32;
    'f16' -> FP16 rounding (via FP32, NumPy's conversion) held in float32.
    """
    g = normal_matrix(k2, k, seed, stream="G", dtype=np.float64,
                      scale=1.0 / math.sqrt(k2))
    if dtype == "f64":
        return g
    if dtype == "f32":
        return np.asfortranarray(g.astype(np.float32))
    if dtype == "bf16":
        return np.asfortranarray(to_bf16_values(g.astype(np.float32)))
    if dtype == "f16":
        return np.asfortranarray(g.astype(np.float32).astype(np.float16).astype(np.float32))
    raise ValueError(dtype)


def orthogonal(n: int, seed: int) -> np.ndarray:
    """Q from the QR factorisation of an n x n Gaussian (LAPACK's output as is)."""
    m = normal_matrix(n, n, seed, stream="Q")
    q, _ = np.linalg.qr(m)
    return np.asfortranarray(q)


def conditioned_matrix(d: int, n: int, kappa: float, seed: int, dtype=np.float64,
                       rotate: bool = True) -> np.ndarray:
    """A = Z diag(logspace(0, -log10 kappa, n)) [Q], Z i.i.d. N(0,1) (FP64),
    rounded to ``dtype``.  Condition number about kappa when rotated."""
    Z = normal_matrix(d, n, seed, stream="A", dtype=np.float64)
    dvec = np.logspace(0.0, -math.log10(kappa), n) if n > 1 else np.ones(1)
    if rotate:
        M = dvec[:, None] * orthogonal(n, seed)
        out = np.empty((d, n), dtype=np.dtype(dtype), order="F")
        step = 1 << 18
        for r0 in range(0, d, step):
            out[r0:r0 + step] = Z[r0:r0 + step] @ M
        return out
    Z *= dvec[None, :]
    return np.asfortranarray(Z.astype(dtype, copy=False))


def lstsq_rhs(A: np.ndarray, nrhs: int, seed: int, noise: float = 1e-6,
              dtype=None):
    """B = A x* + noise * N(0,1), x* ~ N(0,1) (n x nrhs); computed in FP64
    and rounded to A's dtype (or ``dtype``).  Returns (B, xstar)."""
    d, n = A.shape
    xs = normal_matrix(n, nrhs, seed, stream="xstar")
    B = np.empty((d, nrhs), dtype=np.float64, order="F")
    step = 1 << 18
    for r0 in range(0, d, step):
        B[r0:r0 + step] = A[r0:r0 + step].astype(np.float64) @ xs
    if noise:
        B += noise * normal_matrix(d, nrhs, seed, stream="noise")
    out_dtype = np.dtype(dtype) if dtype is not None else A.dtype
    return np.asfortranarray(B.astype(out_dtype, copy=False)), xs


def paper_rhs(A: np.ndarray, seed: int, mu: float = 0.0, sigma2: float = 0.0):
    """b = A e + eta, eta_i ~ N(mu, sigma2), e the all-ones vector (Sec. 6.3's
    easy/hard problems; sigma2 = 0 gives the consistent b = A e)."""
    d, n = A.shape
    b = A.astype(np.float64) @ np.ones(n)
    if sigma2 > 0 or mu != 0:
        b += mu + math.sqrt(sigma2) * normal_matrix(d, 1, seed, stream="noise")[:, 0]
    return np.asfortranarray(b.reshape(d, 1).astype(A.dtype))


# --------------------------------------------------------------------------
# Named workloads (sizes of the five configurations this project targets)
# --------------------------------------------------------------------------

WORKLOADS = {
    "countsketch_65536x32_f64_k2048": dict(d=65536, n=32, k=2048, dtype="f64"),
    "multisketch_lstsq_4194304x64_f64_k8192_k2_128": dict(
        d=4194304, n=64, nrhs=1, k=8192, k2=128, dtype="f64", g_dtype="f64"),
    "multisketch_lstsq_16777216x128_f32_k32768_k2_256_kappa1e6": dict(
        d=16777216, n=128, nrhs=1, k=32768, k2=256, dtype="f32", g_dtype="f32",
        kappa=1e6),
    "mixed_lstsq_8388608x256_f32_k131072_k2_512_bf16": dict(
        d=8388608, n=256, nrhs=4, k=131072, k2=512, dtype="f32", g_dtype="bf16",
        colscale=1e-4, refine=3),
}


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    g = _gen(seed, STREAM["arrivals"])
    return np.cumsum(g.exponential(1.0 / rate, size=count))


def serving_requests(count: int, seed: int, d_lo: int = 1 << 14, d_hi: int = 1 << 20,
                     ns=(8, 16, 32, 64, 128), nrhs_max: int = 8,
                     kappa_lo: float = 1e1, kappa_hi: float = 1e5):
    """Request descriptors of the serving stream: d log-uniform in [d_lo, d_hi],
    n uniform over ``ns``, RHS count uniform in 1..nrhs_max, condition number
    log-uniform in [kappa_lo, kappa_hi]; k = 2 n^2, k2 = 2 n."""
    g = _gen(seed, STREAM["req"])
    lo, hi = math.log2(d_lo), math.log2(d_hi)
    out = []
    for r in range(count):
        d = int(2.0 ** g.uniform(lo, hi))
        n = int(ns[int(g.integers(0, len(ns)))])
        nrhs = int(g.integers(1, nrhs_max + 1))
        kappa = float(10.0 ** g.uniform(math.log10(kappa_lo), math.log10(kappa_hi)))
        out.append(dict(id=r, d=d, n=n, nrhs=nrhs, kappa=kappa, k=2 * n * n,
                        k2=2 * n, seed=int(seed) * 1000003 + r))
    return out
