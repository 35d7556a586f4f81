"""CPU oracle for the CountSketch -> multisketch -> sketch-and-solve path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports,
links or runs anything in this directory, and this directory imports nothing
from the product package.

The arithmetic lives in ``oracle.c`` (plain C, built with
``-O2 -ffp-contract=off -fno-fast-math``); this module only marshals NumPy
arrays (column-major, i.e. Fortran order) into it.  Each wrapper names the
passage of the paper (Higgins, Boman, Yamazaki, arXiv 2508.14209) it follows.

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against values fixed by the paper's definitions and by mathematics (dense-S
brute force, invariants, closed forms, special cases, LAPACK cross-checks);
nothing here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# A test that plants a mistake in the oracle points this at a mutant build.
_LIB_PATH = os.environ.get("MSKETCH_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_RANGE, ERR_NOMEM, ERR_SINGULAR = 0, 1, 2, 3, 4

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC",
          "-shared"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        sig = {
            "or_countsketch_f64": [_i64, _i64, _i64, _p, _i64, _p, _p, _p, _i64],
            "or_countsketch_f32": [_i64, _i64, _i64, _p, _i64, _p, _p, _p, _i64],
            "or_countsketch_f32_acc64": [_i64, _i64, _i64, _p, _i64, _p, _p, _p, _i64],
            "or_countsketch_f64_cols": [_i64, _i64, _i64, _p, _i64, _p, _p, _p, _i64,
                                        ctypes.c_int],
            "or_bucket_hist": [_i64, _i64, _p, _p],
            "or_bucket_plan": [_i64, _i64, _p, _p, _p],
            "or_gemm_f64": [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64],
            "or_householder_qr": [_i64, _i64, _p, _i64, _p],
            "or_apply_qt": [_i64, _i64, _i64, _p, _i64, _p, _p, _i64],
            "or_trsv_upper": [_i64, _i64, _p, _i64, _p, _i64],
            "or_qr_solve": [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64],
            "or_normal_equations": [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64],
            "or_sketch_lstsq_f64": [_i64, _i64, _i64, _i64, _i64, _p, _i64, _p,
                                    _i64, _p, _p, _p, _i64, _p, _i64, _p, _p],
            "or_sketch_lstsq_f32": [_i64, _i64, _i64, _i64, _i64, _p, _i64, _p,
                                    _i64, _p, _p, _p, _i64, ctypes.c_int, _p,
                                    _i64, _p, _p],
            "or_round_bf16": [ctypes.c_float],
            "or_round_bf16_array": [_i64, _p, _p],
            "or_round_f16": [ctypes.c_float],
            "or_f16_col_exp": [_i64, _p],
            "or_round_f16_colscaled": [_i64, _i64, _p, _i64, _p, _i64],
            "or_rand_cholqr_from_sketch": [_i64, _i64, _i64, _i64, _p, _i64, _p, _i64,
                                           _p, _i64, _p, _i64, _p, _i64],
            "or_splitmix64": [ctypes.c_uint64, _i64, _p],
            "or_hash_sketch": [_i64, _i64, ctypes.c_uint64, _p, _p],
            "or_srht": [_i64, _i64, _i64, _p, _i64, _p, _p, _p, _i64],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.or_gemm_f64.restype = None
        lib.or_householder_qr.restype = None
        lib.or_apply_qt.restype = None
        lib.or_round_bf16.restype = ctypes.c_float
        lib.or_round_bf16_array.restype = None
        lib.or_round_f16.restype = ctypes.c_float
        lib.or_round_f16_colscaled.restype = None
        lib.or_splitmix64.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _fortran(a, dtype):
    a = np.asarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return np.asfortranarray(a, dtype=dtype)


def _ld(a: np.ndarray) -> int:
    return max(1, a.shape[0])


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed with oracle status %d" % (what, code))
        self.code = code


def _check(code: int, what: str):
    if code != OK:
        raise OracleError(code, what)


# --------------------------------------------------------------------------
# CountSketch: Def. 3, Eq. (2), Alg. 2
# --------------------------------------------------------------------------

def countsketch(A, h, s, k: int, acc: str | None = None, threads: int = 1) -> np.ndarray:
    """Y = S A, S the CountSketch with buckets h (0-based) and signs s (+-1).

    Canonical fold: for each bucket, rows are added in ascending row order
    starting from +0.0, in the accumulation precision (A's own precision unless
    ``acc='f64'`` for an FP32 A).  Def. 3 and Eq. (2); the add-or-subtract form
    of Alg. 2.  ``threads`` > 1 (FP64 A): the same fold with the columns split
    over that many host threads (bit-identical; for timing on all cores).
    """
    A = np.asarray(A)
    lib = _load()
    h = np.ascontiguousarray(h, dtype=np.int32)
    s = np.ascontiguousarray(s, dtype=np.int8)
    if A.dtype == np.float64:
        A = _fortran(A, np.float64)
        d, n = A.shape
        Y = np.zeros((k, n), dtype=np.float64, order="F")
        if threads > 1:
            rc = lib.or_countsketch_f64_cols(d, n, k, _ptr(A), _ld(A), _ptr(h), _ptr(s),
                                             _ptr(Y), max(1, k), int(threads))
        else:
            rc = lib.or_countsketch_f64(d, n, k, _ptr(A), _ld(A), _ptr(h), _ptr(s),
                                        _ptr(Y), max(1, k))
    elif A.dtype == np.float32 and acc == "f64":
        A = _fortran(A, np.float32)
        d, n = A.shape
        Y = np.zeros((k, n), dtype=np.float64, order="F")
        rc = lib.or_countsketch_f32_acc64(d, n, k, _ptr(A), _ld(A), _ptr(h),
                                          _ptr(s), _ptr(Y), max(1, k))
    elif A.dtype == np.float32:
        A = _fortran(A, np.float32)
        d, n = A.shape
        Y = np.zeros((k, n), dtype=np.float32, order="F")
        rc = lib.or_countsketch_f32(d, n, k, _ptr(A), _ld(A), _ptr(h), _ptr(s),
                                    _ptr(Y), max(1, k))
    else:
        raise TypeError("countsketch oracle takes float64 or float32 A")
    if h.shape[0] != d or s.shape[0] != d:
        raise ValueError("h and s must have one entry per row of A")
    _check(rc, "countsketch")
    return Y


def bucket_hist(h, k: int) -> np.ndarray:
    """cnt[m] = #{i : h[i] = m} (the row counts of the buckets of Def. 3)."""
    h = np.ascontiguousarray(h, dtype=np.int32)
    cnt = np.zeros(k, dtype=np.int64)
    _check(_load().or_bucket_hist(h.shape[0], k, _ptr(h), _ptr(cnt)),
           "bucket_hist")
    return cnt


def bucket_plan(h, k: int):
    """(off, perm): exclusive scan of the bucket counts (k+1 entries) and the
    stable counting-sort permutation (rows of each bucket in ascending order)."""
    h = np.ascontiguousarray(h, dtype=np.int32)
    off = np.zeros(k + 1, dtype=np.int64)
    perm = np.zeros(max(1, h.shape[0]), dtype=np.int64)
    _check(_load().or_bucket_plan(h.shape[0], k, _ptr(h), _ptr(off), _ptr(perm)),
           "bucket_plan")
    return off, perm[: h.shape[0]]


# --------------------------------------------------------------------------
# Gaussian stage: Sec. 1 (multisketch S2(S1 x)), Table 1
# --------------------------------------------------------------------------

def gemm(G, Y) -> np.ndarray:
    """Z = G Y in FP64, each entry folded in ascending inner index from +0.0."""
    G = _fortran(G, np.float64)
    Y = _fortran(Y, np.float64)
    M, K = G.shape
    K2, N = Y.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    Z = np.zeros((M, N), dtype=np.float64, order="F")
    _load().or_gemm_f64(M, N, K, _ptr(G), _ld(G), _ptr(Y), _ld(Y), _ptr(Z),
                        max(1, M))
    return Z


# --------------------------------------------------------------------------
# Householder QR, Q^T application, triangular solve: Alg. 1 steps 2-3;
# GeQRF + OrMQR + TRSV as the paper runs them (Sec. 6.1, 6.3)
# --------------------------------------------------------------------------

def householder_qr(W):
    """Return (F, tau): F holds R in its upper triangle and the Householder
    vectors (unit leading entry implied) below it, LAPACK geqr2 convention."""
    F = np.array(_fortran(W, np.float64), order="F", copy=True)
    m, n = F.shape
    tau = np.zeros(max(1, n), dtype=np.float64)
    _load().or_householder_qr(m, n, _ptr(F), _ld(F), _ptr(tau))
    return F, tau[:n]


def apply_qt(F, tau, B) -> np.ndarray:
    """Q^T B using the reflectors stored in F (what OrMQR computes)."""
    F = _fortran(F, np.float64)
    m, n = F.shape
    Bc = np.array(_fortran(B, np.float64), order="F", copy=True)
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    _load().or_apply_qt(m, n, Bc.shape[1], _ptr(F), _ld(F), _ptr(tau), _ptr(Bc),
                        _ld(Bc))
    return Bc


def trsv_upper(R, B) -> np.ndarray:
    """X with R X = B for the upper triangle of R (n x n); B is n x nrhs."""
    R = _fortran(R, np.float64)
    X = np.array(_fortran(B, np.float64), order="F", copy=True)
    rc = _load().or_trsv_upper(R.shape[1], X.shape[1], _ptr(R), _ld(R), _ptr(X),
                               _ld(X))
    _check(rc, "trsv_upper")
    return X


def qr_solve(W, B) -> np.ndarray:
    """X = R^{-1} (Q^T B)_{0:n} with [Q,R] = qr(W,0) (Alg. 1 steps 2-3)."""
    W = _fortran(W, np.float64)
    B = _fortran(B, np.float64)
    m, n = W.shape
    X = np.zeros((n, B.shape[1]), dtype=np.float64, order="F")
    rc = _load().or_qr_solve(m, n, B.shape[1], _ptr(W), _ld(W), _ptr(B), _ld(B),
                             _ptr(X), max(1, n))
    _check(rc, "qr_solve")
    return X


def lstsq_qr(A, B) -> np.ndarray:
    """The FP64 least-squares optimum x_t = argmin ||B - A x|| by Householder
    QR of the full A (comparator for the residual ratio)."""
    return qr_solve(A, B)


def normal_equations(A, B) -> np.ndarray:
    """FP64 normal equations (Sec. 6.3): Gram A^T A, A^T b, Cholesky R^T R,
    then R^T y = A^T b and R x = y.  Raises OracleError(ERR_SINGULAR) when the
    Cholesky factorisation breaks down."""
    A = _fortran(A, np.float64)
    B = _fortran(B, np.float64)
    d, n = A.shape
    X = np.zeros((n, B.shape[1]), dtype=np.float64, order="F")
    rc = _load().or_normal_equations(d, n, B.shape[1], _ptr(A), _ld(A), _ptr(B),
                                     _ld(B), _ptr(X), max(1, n))
    _check(rc, "normal_equations")
    return X


# --------------------------------------------------------------------------
# Composite multisketch sketch-and-solve (Alg. 1 with S = G C)
# --------------------------------------------------------------------------

def sketch_lstsq(A, B, h, s, G, k: int, y_bf16: bool = False, y_acc64: bool = False,
                 y_f16: bool = False):
    """X = argmin ||G C (B - A X)|| via Alg. 1 with the multisketch S = G C.

    FP64 A: CountSketch in FP64.  FP32 A: CountSketch in FP32 (folded in FP32
    in the canonical order, or with ``y_acc64`` Def. 3's sums taken in FP64
    and rounded once to FP32), optional RNE rounding of the sketch to BF16
    (``y_bf16``) or to FP16 after the FP16 stage's per-column power-of-two
    scale (``y_f16``, see ``round_f16_colscaled``), Gaussian stage and QR in
    FP64 on the exact FP64 images of the stored values.  G is passed as its
    stored values (float64, float32 or BF16 values held in float32/float64).
    Returns (X, Y, Z): solution n x nrhs, CountSketch k x (n+nrhs) and the
    Gaussian-stage output k2 x (n+nrhs).
    """
    A = np.asarray(A)
    lib = _load()
    h = np.ascontiguousarray(h, dtype=np.int32)
    s = np.ascontiguousarray(s, dtype=np.int8)
    Gd = _fortran(G, np.float64)
    k2 = Gd.shape[0]
    if Gd.shape[1] != k:
        raise ValueError("G must be k2 x k")
    if A.dtype == np.float64:
        A = _fortran(A, np.float64)
        B = _fortran(B, np.float64)
        d, n = A.shape
        nrhs = B.shape[1]
        X = np.zeros((n, nrhs), dtype=np.float64, order="F")
        Y = np.zeros((k, n + nrhs), dtype=np.float64, order="F")
        Z = np.zeros((k2, n + nrhs), dtype=np.float64, order="F")
        rc = lib.or_sketch_lstsq_f64(d, n, nrhs, k, k2, _ptr(A), _ld(A), _ptr(B),
                                     _ld(B), _ptr(h), _ptr(s), _ptr(Gd), _ld(Gd),
                                     _ptr(X), max(1, n), _ptr(Y), _ptr(Z))
    elif A.dtype == np.float32:
        A = _fortran(A, np.float32)
        B = _fortran(B, np.float32)
        d, n = A.shape
        nrhs = B.shape[1]
        X = np.zeros((n, nrhs), dtype=np.float64, order="F")
        Y = np.zeros((k, n + nrhs), dtype=np.float32, order="F")
        Z = np.zeros((k2, n + nrhs), dtype=np.float64, order="F")
        rc = lib.or_sketch_lstsq_f32(d, n, nrhs, k, k2, _ptr(A), _ld(A), _ptr(B),
                                     _ld(B), _ptr(h), _ptr(s), _ptr(Gd), _ld(Gd),
                                     (1 if y_bf16 else 0) | (2 if y_acc64 else 0) |
                                     (4 if y_f16 else 0),
                                     _ptr(X), max(1, n),
                                     _ptr(Y), _ptr(Z))
    else:
        raise TypeError("sketch_lstsq oracle takes float64 or float32 A")
    if rc == ERR_SINGULAR:
        return X, Y, Z
    _check(rc, "sketch_lstsq")
    return X, Y, Z


# --------------------------------------------------------------------------
# rand_cholQR least squares (Alg. 5) with the multisketch S = G C
# --------------------------------------------------------------------------

def rand_cholqr_from_sketch(SA, A, B):
    """Alg. 5 steps 2-8 given the sketch SA = S A (m x n): R0 from the
    Householder QR of SA, Q0 = A R0^{-1} row by row, Gm = Q0^T Q0 and
    z = Q0^T B, R1 = chol(Gm), R = R1 R0, y = R1^{-T} z, x = R^{-1} y, all in
    FP64 (an FP32 A or B is promoted exactly).  Returns (X, R)."""
    SA = _fortran(SA, np.float64)
    A = _fortran(A, np.float64)
    B = _fortran(B, np.float64)
    m, n = SA.shape
    d = A.shape[0]
    nrhs = B.shape[1]
    X = np.zeros((n, nrhs), dtype=np.float64, order="F")
    R = np.zeros((n, n), dtype=np.float64, order="F")
    rc = _load().or_rand_cholqr_from_sketch(d, n, nrhs, m, _ptr(SA), _ld(SA), _ptr(A), _ld(A),
                                            _ptr(B), _ld(B), _ptr(X), max(1, n), _ptr(R),
                                            max(1, n))
    _check(rc, "rand_cholqr")
    return X, R


def rand_cholqr_lstsq(A, B, h, s, G, k: int, y_bf16: bool = False, y_f16: bool = False):
    """x = argmin ||B - A x|| by rand_cholQR least squares (Alg. 5) with the
    multisketch S = G C as the sketch operator (step 1: the CountSketch of A
    in A's precision, optionally rounded to BF16 for an FP32 A, then the
    Gaussian stage in FP64 on the stored values of G).  Returns (X, R, SA)."""
    A = np.asarray(A)
    Gd = _fortran(G, np.float64)
    if Gd.shape[1] != k:
        raise ValueError("G must be k2 x k")
    Y = countsketch(A, h, s, k)
    if A.dtype == np.float32 and y_bf16:
        Y = round_bf16(Y)
    elif A.dtype == np.float32 and y_f16:
        Y = round_f16_colscaled(Y)
    SA = gemm(Gd, np.asarray(Y, dtype=np.float64))
    X, R = rand_cholqr_from_sketch(SA, A, B)
    return X, R, SA


# --------------------------------------------------------------------------
# Hash-generated CountSketch (Sec. 8, future work): (h, s) from SplitMix64
# --------------------------------------------------------------------------

def splitmix64(seed: int, count: int) -> np.ndarray:
    """``count`` successive outputs of SplitMix64 started at state ``seed``
    (Steele, Lea and Flood, OOPSLA 2014), as uint64."""
    out = np.zeros(int(count), dtype=np.uint64)
    _load().or_splitmix64(ctypes.c_uint64(int(seed) & (2**64 - 1)), int(count), _ptr(out))
    return out


def hash_sketch(d: int, k: int, seed: int):
    """Bucket map h (int32) and signs s (int8) of the hash-generated
    CountSketch: row i takes u = the (i+1)-th SplitMix64 output from state
    ``seed``; h = floor((u >> 32) k / 2^32), s = -1 if bit 0 of u else +1."""
    h = np.zeros(int(d), dtype=np.int32)
    s = np.zeros(int(d), dtype=np.int8)
    _check(_load().or_hash_sketch(int(d), int(k), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                  _ptr(h), _ptr(s)), "hash_sketch")
    return h, s


def countsketch_hashed(A, k: int, seed: int, acc: str | None = None) -> np.ndarray:
    """Y = C A for the CountSketch C whose (h, s) are ``hash_sketch(d, k,
    seed)`` (Def. 3 with generated instead of stored vectors)."""
    A = np.asarray(A)
    h, s = hash_sketch(A.shape[0], k, seed)
    return countsketch(A, h, s, k, acc=acc)


# --------------------------------------------------------------------------
# SRHT (Sec. 5) and the Count + SRHT multisketch (Sec. 8, future work)
# --------------------------------------------------------------------------

def srht(X, dsign, r) -> np.ndarray:
    """Y = k^{-1/2} P H_m D X (k x ncols, FP64) by the SRHT's definition:
    H_m[a][b] = (-1)^popcount(a & b), m = the smallest power of two >= the
    rows of X (zero rows appended), D = diag(dsign) (+-1, one per row of X),
    P taking rows r (k int32 in [0, m)) of H_m D X."""
    X = _fortran(X, np.float64)
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    mx, nc = X.shape
    dsign = np.ascontiguousarray(dsign, dtype=np.int8)
    r = np.ascontiguousarray(r, dtype=np.int32)
    k = r.shape[0]
    Y = np.zeros((k, nc), dtype=np.float64, order="F")
    _check(_load().or_srht(mx, nc, k, _ptr(X), _ld(X), _ptr(dsign), _ptr(r), _ptr(Y),
                           max(1, k)), "srht")
    return Y


def count_srht_sketch(A, h, s, k1: int, dsign, r, acc: str | None = None) -> np.ndarray:
    """The Count + SRHT multisketch S2 (C A): the CountSketch of A (k1
    buckets, A's precision) followed by the SRHT (FP64) of its k1 rows."""
    Y = countsketch(A, h, s, k1, acc=acc)
    return srht(np.asarray(Y, dtype=np.float64), dsign, r)


def count_srht_lstsq(A, B, h, s, k1: int, dsign, r):
    """Alg. 1 with the Count + SRHT multisketch as S: Z = S [A | B] (C in A's
    precision, the SRHT and the QR least squares in FP64).  Returns X."""
    A = np.asarray(A)
    B = np.asarray(B)
    if B.ndim == 1:
        B = B[:, None]
    n = A.shape[1]
    AB = np.asfortranarray(np.concatenate([A, B.astype(A.dtype)], axis=1))
    Z = count_srht_sketch(AB, h, s, k1, dsign, r)
    return qr_solve(Z[:, :n], Z[:, n:])


def round_bf16(x) -> np.ndarray:
    """Round FP32 values to BF16 (RNE), returned as the FP32 values they are."""
    lib = _load()
    x = np.asarray(x, dtype=np.float32)
    order = "F" if x.flags.f_contiguous and not x.flags.c_contiguous else "C"
    flat = np.ascontiguousarray(x.reshape(-1, order=order))
    out = np.empty_like(flat)
    lib.or_round_bf16_array(flat.shape[0], _ptr(flat), _ptr(out))
    return out.reshape(x.shape, order=order)


def round_f16(x) -> np.ndarray:
    """Round FP32 values to FP16 (IEEE binary16, RNE, subnormals kept,
    overflow to infinity), returned as the FP32 values they are."""
    lib = _load()
    x = np.asarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.float32)
    flat_in = x.reshape(-1)
    flat_out = out.reshape(-1)
    for i in range(flat_in.shape[0]):
        flat_out[i] = lib.or_round_f16(float(flat_in[i]))
    return out


def f16_col_exp(y) -> int:
    """The FP16 Gaussian stage's scale exponent of one FP32 column:
    floor(log2 max |y|) - 14 held in [-112, 112]; 0 for a zero or
    non-finite column."""
    y = np.ascontiguousarray(y, dtype=np.float32).reshape(-1)
    return int(_load().or_f16_col_exp(y.shape[0], _ptr(y)))


def round_f16_colscaled(Y) -> np.ndarray:
    """Y (k x nc, FP32) as the FP16 Gaussian stage reads it: column c scaled
    by 2^-e_c (e_c = f16_col_exp of the column; an FP32 product), rounded to
    FP16 (RNE) and scaled back by 2^e_c.  Returns FP64 (exact values)."""
    Y = _fortran(Y, np.float32)
    if Y.ndim == 1:
        Y = Y.reshape(-1, 1, order="F")
    k, nc = Y.shape
    out = np.zeros((k, nc), dtype=np.float64, order="F")
    _load().or_round_f16_colscaled(k, nc, _ptr(Y), _ld(Y), _ptr(out), max(1, k))
    return out


def lstsq_tsqr(A, B, block_rows: int = 1 << 18):
    """The FP64 least-squares optimum of min ||B - A X|| for tall A that need
    not fit in memory twice: Householder QR of [A | B] taken over blocks of
    rows (each block stacked under the running triangular factor and
    re-factored, LAPACK's QR as the step), giving
        [A | B] = Q [[R11, R12], [0, R22]],  X = R11^{-1} R12,
        ||B[:, j] - A X[:, j]|| = ||R22[:, j]||.
    A is promoted to FP64 block by block.  Returns (X, residual norms)."""
    A = np.asarray(A)
    B = np.asarray(B)
    if B.ndim == 1:
        B = B[:, None]
    d, n = A.shape
    nrhs = B.shape[1]
    R = np.zeros((0, n + nrhs))
    for r0 in range(0, d, block_rows):
        blk = np.empty((min(d, r0 + block_rows) - r0, n + nrhs))
        blk[:, :n] = A[r0:r0 + block_rows]
        blk[:, n:] = B[r0:r0 + block_rows]
        R = np.linalg.qr(np.vstack([R, blk]), mode="r")
    R11, R12 = R[:n, :n], R[:n, n:]
    R22 = R[n:, n:]
    X = np.linalg.solve(np.triu(R11), R12) if n else np.zeros((0, nrhs))
    res = np.array([np.linalg.norm(R22[:, j]) for j in range(nrhs)])
    return X, res
