"""msketch: MI355X-native CountSketch, multisketch and sketch-and-solve least
squares (Higgins, Boman, Yamazaki, arXiv 2508.14209).

Thin Python binding of the C ABI in ``include/msketch.h`` (``libmsketch.so``):
every function here only checks shapes, takes device pointers, leading
dimensions and the current HIP stream from torch tensors, and calls the entry
point of the same name.  All arithmetic runs in the library's HIP kernels.
There is no CPU fallback: importing this module without the built library
raises.

Matrices are column-major (``t.stride(0) == 1``); ``empty_colmajor`` makes
such tensors.  BF16 Gaussian matrices are ``torch.bfloat16`` tensors.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "MS_OK", "MS_ERR_ARG", "MS_ERR_RANGE", "MS_ERR_NOMEM", "MS_ERR_SINGULAR",
    "MS_ERR_DEVICE", "MS_ERR_UNSUPPORTED", "MsketchError", "LIB_PATH",
    "empty_colmajor", "colmajor", "workspace", "workspace_size", "check_status",
    "bucket_plan", "pack_sketch", "countsketch_accumulate", "countsketch_apply",
    "gaussian_apply", "multisketch_apply", "qr_solve", "sketch_lstsq", "sketch_lstsq_noalloc",
    "NOALLOC_SCRATCH_BYTES", "rand_cholqr_lstsq",
    "normal_equations_lstsq", "countsketch_hashed", "hash_sketch", "srht_apply",
    "count_srht_lstsq", "MsProblem",
    "batch_workspace_size", "sketch_lstsq_batched", "batch_status", "BatchRunner",
    "gen_lstsq_request",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsketch.so")

MS_OK, MS_ERR_ARG, MS_ERR_RANGE, MS_ERR_NOMEM, MS_ERR_SINGULAR, MS_ERR_DEVICE, \
    MS_ERR_UNSUPPORTED = range(7)
MS_F64, MS_F32, MS_BF16, MS_F16 = 0, 1, 2, 3
MODES = {"auto": 0, "atomic": 1, "lds": 2, "sorted": 3}
OPS = {"bucket_plan": 0, "countsketch": 1, "gaussian": 2, "multisketch": 3,
       "qr_solve": 4, "lstsq": 5, "rand_cholqr": 6,
       "normal_equations": 7, "countsketch_hashed": 8, "srht": 9,
       "count_srht_lstsq": 10}
MS_SORTED_MAX_SEGMENT = 16384
MS_SORTED_BLOCKED_MAX_K = 16384
NOALLOC_SCRATCH_BYTES = 32 << 20   # MS_NOALLOC_SCRATCH_BYTES of msketch.h

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libmsketch.so is not built (%s); run `python paper_2508_14209_amd/build.py` "
        "or __graft_entry__.build()" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)
_i64, _p, _sz, _i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int


class MsOpts(ctypes.Structure):
    _fields_ = [("cs_mode", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("cs_tile_cols", ctypes.c_int32), ("cs_schedule", ctypes.c_int32),
                ("batch_rows_log2", ctypes.c_int32), ("batch_kchunk_log2", ctypes.c_int32),
                ("gauss_y_terms", ctypes.c_int32), ("refine_tol_log2", ctypes.c_int32)]


class MsProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int64), ("n", ctypes.c_int64), ("nrhs", ctypes.c_int64),
                ("k", ctypes.c_int64), ("k2", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("h", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("G", ctypes.c_void_p), ("ldg", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64)]


_SIGS = {
    "ms_workspace_size": ([_i32, _i64, _i64, _i64, _i64, _i64, _i32, _i32, _p], _sz),
    "ms_check_status": ([_p, _p], _i32),
    "ms_status_string": ([_i32], ctypes.c_char_p),
    "ms_bucket_plan": ([_i64, _i64, _p, _p, _p, _p, _p, _sz, _p], _i32),
    "ms_pack_sketch": ([_i64, _i64, _p, _p, _p, _p, _sz, _p], _i32),
    "countsketch_accumulate": ([_i64, _i64, _i64, _i32, _p, _i64, _p, _p, _i64, _p, _p, _sz,
                                _p], _i32),
    "countsketch_apply": ([_i64, _i64, _i64, _i32, _p, _i64, _p, _p, _p, _i64, _p, _p,
                           _sz, _p], _i32),
    "ms_gaussian_apply": ([_i64, _i64, _i64, _i32, _p, _i64, _i32, _p, _i64, _p, _i64,
                           _p, _sz, _p], _i32),
    "multisketch_apply": ([_i64, _i64, _i64, _i64, _i32, _p, _i64, _p, _p, _i32, _p,
                           _i64, _p, _i64, _p, _p, _sz, _p], _i32),
    "ms_qr_solve": ([_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _sz,
                     _p], _i32),
    "sketch_lstsq": ([_i64, _i64, _i64, _i64, _i64, _i32, _p, _i64, _p, _i64, _p, _p,
                      _i32, _p, _i64, _p, _i64, _p, _p, _sz, _p], _i32),
    "sketch_lstsq_noalloc": ([_i64, _i64, _i64, _i64, _i64, _i32, _p, _i64, _p, _i64, _p, _p,
                              _i32, _p, _i64, _p, _i64, _p, _p, _p], _i32),
    "rand_cholqr_lstsq": ([_i64, _i64, _i64, _i64, _i64, _i32, _p, _i64, _p, _i64, _p, _p,
                           _i32, _p, _i64, _p, _i64, _p, _i64, _p, _p, _sz, _p], _i32),
    "normal_equations_lstsq": ([_i64, _i64, _i64, _i32, _p, _i64, _p, _i64, _p, _i64, _p, _i64,
                                _p, _p, _sz, _p], _i32),
    "countsketch_hashed": ([_i64, _i64, _i64, ctypes.c_uint64, _i32, _p, _i64, _p, _i64, _p, _p,
                            _sz, _p], _i32),
    "ms_hash_sketch": ([_i64, _i64, ctypes.c_uint64, _p, _p, _p], _i32),
    "srht_apply": ([_i64, _i64, _i64, _i32, _p, _i64, _p, _p, _p, _i64, _p, _sz, _p], _i32),
    "count_srht_lstsq": ([_i64, _i64, _i64, _i64, _i64, _i32, _p, _i64, _p, _i64, _p, _p, _p, _p,
                          _p, _i64, _p, _p, _sz, _p], _i32),
    "ms_batch_workspace_size": ([_i32, _p, _i32, _i32, _p], _sz),
    "sketch_lstsq_batched": ([_i32, _p, _p, _i32, _i32, _p, _p, _sz, _p], _i32),
    "ms_batch_status": ([_p, _i32, _p, _p], _i32),
    "ms_gen_lstsq_request": ([ctypes.c_uint64, _i64, _i64, _i64, ctypes.c_double, ctypes.c_double,
                              _i64, _i64, _i32, _p, _i64, _p, _i64, _p, _p, _p, _p, _p], _i32),
}
for _name, (_args, _ret) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _ret


class MsketchError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.ms_status_string(code).decode()
        super().__init__("%s: %s" % (where, msg))
        self.code = code


def _ok(code: int, where: str):
    if code != MS_OK:
        raise MsketchError(code, where)


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return MS_F64
    if t.dtype == torch.float32:
        return MS_F32
    if t.dtype == torch.bfloat16:
        return MS_BF16
    if t.dtype == torch.float16:
        return MS_F16
    raise TypeError("unsupported dtype %s" % t.dtype)


_TORCH_DT = {MS_F64: torch.float64, MS_F32: torch.float32, MS_BF16: torch.bfloat16,
             MS_F16: torch.float16}


def empty_colmajor(rows: int, cols: int, dtype, device="cuda") -> torch.Tensor:
    """A rows x cols tensor in column-major storage (leading dimension rows)."""
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def colmajor(t: torch.Tensor, name: str):
    """(pointer, leading dimension) of a 2-D column-major device tensor."""
    if t.dim() == 1:
        t = t.unsqueeze(1)
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    rows, cols = t.shape
    if rows > 1 and t.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1)" % name)
    ld = t.stride(1) if cols > 1 else max(1, rows)
    return t.data_ptr(), max(ld, rows, 1)


def _vec(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda or t.dtype != dtype or t.dim() != 1 or (t.numel() > 1 and t.stride(0) != 1):
        raise ValueError("%s must be a contiguous 1-D %s device tensor" % (name, dtype))
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _opts(mode: str = "auto", refine_steps: int = 0, tile_cols: int = 0, schedule: int = 0,
          rows_log2: int = 0, kchunk_log2: int = 0, y_terms: int = 0, refine_tol_log2: int = 0):
    return MsOpts(MODES[mode], int(refine_steps), int(tile_cols), int(schedule), int(rows_log2),
                  int(kchunk_log2), int(y_terms), int(refine_tol_log2))


def workspace_size(op: str, d=0, n=0, nrhs=0, k=0, k2=0, a_dtype=MS_F64, g_dtype=MS_F64,
                   mode: str = "auto", refine_steps: int = 0) -> int:
    o = _opts(mode, refine_steps)
    sz = _lib.ms_workspace_size(OPS[op], d, n, nrhs, k, k2, a_dtype, g_dtype, ctypes.byref(o))
    if sz == 0:
        raise MsketchError(MS_ERR_ARG, "ms_workspace_size")
    return sz


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """A device byte buffer usable as a workspace (256-byte aligned)."""
    return torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)


def _ws_ptr(ws: torch.Tensor, need: int):
    p = ws.data_ptr()
    aligned = (p + 255) // 256 * 256
    have = ws.numel() - (aligned - p)
    if have < need:
        raise MsketchError(MS_ERR_NOMEM, "workspace")
    return aligned, have


def check_status(ws: torch.Tensor, stream=None, where: str = "device status"):
    """Synchronise and raise MsketchError if the last call that used ``ws``
    recorded a device-side error."""
    p = (ws.data_ptr() + 255) // 256 * 256
    _ok(_lib.ms_check_status(ctypes.c_void_p(p), _stream(stream)), where)


def bucket_plan(h: torch.Tensor, k: int, ws: torch.Tensor | None = None, stream=None):
    """(cnt, off, perm) of the stable counting sort of rows by bucket."""
    d = h.numel()
    need = workspace_size("bucket_plan", d=d, k=k)
    ws = workspace(need, h.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    cnt = torch.empty(k, dtype=torch.int32, device=h.device)
    off = torch.empty(k + 1, dtype=torch.int32, device=h.device)
    perm = torch.empty(max(d, 1), dtype=torch.int32, device=h.device)
    _ok(_lib.ms_bucket_plan(d, k, _vec(h, torch.int32, "h") if d else None, cnt.data_ptr(),
                            off.data_ptr(), perm.data_ptr(), wp, have, _stream(stream)),
        "ms_bucket_plan")
    return cnt, off, perm[:d], ws


def pack_sketch(h: torch.Tensor, s: torch.Tensor, k: int, code: torch.Tensor | None = None,
                ws: torch.Tensor | None = None, stream=None):
    """Validated packed sketch: one int32 word per row, h | (s == -1) << 31.
    Returns (code, ws)."""
    d = h.numel()
    if code is None:
        code = torch.empty(max(d, 1), dtype=torch.int32, device=h.device)
    ws = workspace(256, h.device) if ws is None else ws
    wp, have = _ws_ptr(ws, 256)
    _ok(_lib.ms_pack_sketch(d, k, _vec(h, torch.int32, "h") if d else None,
                            _vec(s, torch.int8, "s") if d else None,
                            code.data_ptr(), wp, have, _stream(stream)), "ms_pack_sketch")
    return code[:d], ws


def countsketch_accumulate(A: torch.Tensor, code: torch.Tensor, k: int, Y: torch.Tensor,
                           mode: str = "auto", ws: torch.Tensor | None = None, stream=None,
                           tile_cols: int = 0, schedule: int = 0):
    """Y += S A with a packed sketch (no clearing of Y).  Returns (Y, ws)."""
    d, n = A.shape
    a_dt = _dt(A)
    Ap, lda = colmajor(A, "A")
    Yp, ldy = colmajor(Y, "Y")
    if Y.shape != (k, n) or Y.dtype != A.dtype:
        raise ValueError("Y must be k x n with A's dtype")
    ws = workspace(256, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, 256)
    o = _opts(mode, 0, tile_cols, schedule)
    _ok(_lib.countsketch_accumulate(d, n, k, a_dt, Ap, lda,
                                    _vec(code, torch.int32, "code") if d else None, Yp, ldy,
                                    ctypes.byref(o), wp, have, _stream(stream)),
        "countsketch_accumulate")
    return Y, ws


def countsketch_apply(A: torch.Tensor, h: torch.Tensor, s: torch.Tensor, k: int,
                      Y: torch.Tensor | None = None, mode: str = "auto",
                      ws: torch.Tensor | None = None, stream=None, tile_cols: int = 0,
                      schedule: int = 0):
    """Y = S A (k x n, A's dtype).  Returns (Y, ws)."""
    d, n = A.shape
    a_dt = _dt(A)
    Ap, lda = colmajor(A, "A")
    if Y is None:
        Y = empty_colmajor(k, n, A.dtype, A.device)
    Yp, ldy = colmajor(Y, "Y")
    if Y.shape != (k, n) or Y.dtype != A.dtype:
        raise ValueError("Y must be k x n with A's dtype")
    need = workspace_size("countsketch", d=d, n=n, k=k, a_dtype=a_dt, mode=mode)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    o = _opts(mode, 0, tile_cols, schedule)
    _ok(_lib.countsketch_apply(d, n, k, a_dt, Ap, lda,
                               _vec(h, torch.int32, "h") if d else None,
                               _vec(s, torch.int8, "s") if d else None, Yp, ldy,
                               ctypes.byref(o), wp, have, _stream(stream)), "countsketch_apply")
    return Y, ws


def countsketch_hashed(A: torch.Tensor, k: int, seed: int, Y: torch.Tensor | None = None,
                       ws: torch.Tensor | None = None, stream=None, tile_cols: int = 0):
    """Y = C A (k x n, A's dtype) for the hash-generated CountSketch: row i's
    bucket and sign come from SplitMix64's (i+1)-th output from state
    ``seed`` (no stored h, s).  Returns (Y, ws)."""
    d, n = A.shape
    a_dt = _dt(A)
    Ap, lda = colmajor(A, "A")
    if Y is None:
        Y = empty_colmajor(k, n, A.dtype, A.device)
    Yp, ldy = colmajor(Y, "Y")
    if Y.shape != (k, n) or Y.dtype != A.dtype:
        raise ValueError("Y must be k x n with A's dtype")
    need = workspace_size("countsketch_hashed", d=d, n=n, k=k, a_dtype=a_dt)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    o = _opts("auto", 0, tile_cols, 0)
    _ok(_lib.countsketch_hashed(d, n, k, int(seed) & (2**64 - 1), a_dt, Ap, lda, Yp, ldy,
                                ctypes.byref(o), wp, have, _stream(stream)), "countsketch_hashed")
    return Y, ws


def gen_lstsq_request(seed: int, d: int, n: int, nrhs: int, kappa: float, k: int, k2: int,
                      g_dtype=MS_F32, noise: float = 1e-6, device="cuda", stream=None,
                      want=("A", "B", "xstar", "h", "s", "G")) -> dict:
    """A seeded synthetic request generated on the device by
    ms_gen_lstsq_request: A = Z diag(kappa^(-j/(n-1))) Q (FP32, column-major),
    B = A xstar + noise N(0,1), h, s, G (k2 x k, column-major, dtype g_dtype)
    = N(0,1)/sqrt(k2).  Only the parts named in `want` are made."""
    out = {}
    if "A" in want or "B" in want:
        out["A"] = empty_colmajor(d, n, torch.float32, device)
    if "B" in want:
        out["B"] = empty_colmajor(d, nrhs, torch.float32, device)
    if "xstar" in want:
        out["xstar"] = empty_colmajor(n, nrhs, torch.float32, device)
    if "h" in want or "s" in want:
        out["h"] = torch.empty(d, dtype=torch.int32, device=device)
        out["s"] = torch.empty(d, dtype=torch.int8, device=device)
    if "G" in want:
        gt = {MS_F32: torch.float32, MS_BF16: torch.bfloat16, MS_F64: torch.float64}[g_dtype]
        out["G"] = empty_colmajor(k2, k, gt, device)

    def ptr(name):
        t = out.get(name)
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    _ok(_lib.ms_gen_lstsq_request(int(seed) & (2**64 - 1), d, n, nrhs, float(kappa), float(noise),
                                  k, k2, int(g_dtype), ptr("A"), d, ptr("B"), d, ptr("xstar"),
                                  ptr("h"), ptr("s"), ptr("G"), _stream(stream)),
        "ms_gen_lstsq_request")
    return out


def hash_sketch(d: int, k: int, seed: int, device="cuda", stream=None):
    """h (int32) and s (int8) of the hash-generated CountSketch, on the device."""
    h = torch.empty(d, dtype=torch.int32, device=device)
    s = torch.empty(d, dtype=torch.int8, device=device)
    _ok(_lib.ms_hash_sketch(d, k, int(seed) & (2**64 - 1), h.data_ptr() if d else None,
                            s.data_ptr() if d else None, _stream(stream)), "ms_hash_sketch")
    return h, s


def srht_apply(X: torch.Tensor, dsign: torch.Tensor, r: torch.Tensor,
               Y: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """Y = k^{-1/2} P H_m D X (k x ncols, FP64): the SRHT with D = diag(dsign)
    and P taking rows r of H_m D X (m = X's rows rounded up to a power of
    two).  Returns (Y, ws)."""
    if X.dim() == 1:
        X = X.unsqueeze(1)
    m, nc = X.shape
    k = r.shape[0]
    x_dt = _dt(X)
    if Y is None:
        Y = empty_colmajor(k, nc, torch.float64, X.device)
    Xp, ldx = colmajor(X, "X")
    Yp, ldy = colmajor(Y, "Y")
    need = workspace_size("srht", d=m, n=nc, k=k, a_dtype=x_dt)
    ws = workspace(need, X.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    _ok(_lib.srht_apply(m, nc, k, x_dt, Xp, ldx, _vec(dsign, torch.int8, "dsign"),
                        _vec(r, torch.int32, "r"), Yp, ldy, wp, have, _stream(stream)),
        "srht_apply")
    return Y, ws


def count_srht_lstsq(A: torch.Tensor, B: torch.Tensor, h: torch.Tensor, s: torch.Tensor,
                     k1: int, dsign: torch.Tensor, r: torch.Tensor, mode: str = "auto",
                     X: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """Sketch-and-solve with the Count + SRHT multisketch: Z = S2 (C [A | B])
    (C: h, s, k1 buckets; S2: the SRHT with dsign, r), then QR least
    squares in FP64.  Returns (X, ws)."""
    d, n = A.shape
    if B.dim() == 1:
        B = B.unsqueeze(1)
    nrhs = B.shape[1]
    k2 = r.shape[0]
    a_dt = _dt(A)
    if B.dtype != A.dtype:
        raise ValueError("B must have A's dtype")
    if X is None:
        X = empty_colmajor(n, nrhs, torch.float64, A.device)
    Ap, lda = colmajor(A, "A")
    Bp, ldb = colmajor(B, "B")
    Xp, ldx = colmajor(X, "X")
    need = workspace_size("count_srht_lstsq", d=d, n=n, nrhs=nrhs, k=k1, k2=k2, a_dtype=a_dt,
                          mode=mode)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    o = _opts(mode, 0)
    _ok(_lib.count_srht_lstsq(d, n, nrhs, k1, k2, a_dt, Ap, lda, Bp, ldb,
                              _vec(h, torch.int32, "h"), _vec(s, torch.int8, "s"),
                              _vec(dsign, torch.int8, "dsign"), _vec(r, torch.int32, "r"), Xp, ldx,
                              ctypes.byref(o), wp, have, _stream(stream)), "count_srht_lstsq")
    return X, ws


def gaussian_apply(G: torch.Tensor, Y: torch.Tensor, Z: torch.Tensor | None = None,
                   ws: torch.Tensor | None = None, stream=None):
    """Z = G Y (k2 x ncols).  Returns (Z, ws)."""
    k2, k = G.shape
    k_, nc = Y.shape
    if k_ != k:
        raise ValueError("G is k2 x k and Y is k x ncols")
    g_dt, y_dt = _dt(G), _dt(Y)
    zdtype = torch.float64 if g_dt == MS_F64 else torch.float32
    if Z is None:
        Z = empty_colmajor(k2, nc, zdtype, Y.device)
    Gp, ldg = colmajor(G, "G")
    Yp, ldy = colmajor(Y, "Y")
    Zp, ldz = colmajor(Z, "Z")
    need = workspace_size("gaussian", n=nc, k=k, k2=k2, a_dtype=y_dt, g_dtype=g_dt)
    ws = workspace(need, Y.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    _ok(_lib.ms_gaussian_apply(k, nc, k2, g_dt, Gp, ldg, y_dt, Yp, ldy, Zp, ldz, wp, have,
                               _stream(stream)), "ms_gaussian_apply")
    return Z, ws


def multisketch_apply(A: torch.Tensor, h: torch.Tensor, s: torch.Tensor, G: torch.Tensor,
                      k: int, Z: torch.Tensor | None = None, mode: str = "auto",
                      ws: torch.Tensor | None = None, stream=None, y_terms: int = 0):
    """Z = G (S A) (k2 x n).  y_terms (BF16 or FP16 G): 1 = S A rounded to G's
    16-bit format (FP16: after a power-of-two scale per column), 3 (or 0, the
    default) = S A as three exact 16-bit terms.  Returns (Z, ws)."""
    d, n = A.shape
    k2 = G.shape[0]
    a_dt, g_dt = _dt(A), _dt(G)
    zdtype = torch.float64 if a_dt == MS_F64 else torch.float32
    if Z is None:
        Z = empty_colmajor(k2, n, zdtype, A.device)
    Ap, lda = colmajor(A, "A")
    Gp, ldg = colmajor(G, "G")
    Zp, ldz = colmajor(Z, "Z")
    need = workspace_size("multisketch", d=d, n=n, k=k, k2=k2, a_dtype=a_dt, g_dtype=g_dt,
                          mode=mode)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    o = _opts(mode, y_terms=y_terms)
    _ok(_lib.multisketch_apply(d, n, k, k2, a_dt, Ap, lda,
                               _vec(h, torch.int32, "h") if d else None,
                               _vec(s, torch.int8, "s") if d else None, g_dt, Gp, ldg, Zp, ldz,
                               ctypes.byref(o), wp, have, _stream(stream)), "multisketch_apply")
    return Z, ws


def qr_solve(W: torch.Tensor, B: torch.Tensor, X: torch.Tensor | None = None,
             R: torch.Tensor | None = None, want_r: bool = False,
             ws: torch.Tensor | None = None, stream=None):
    """X = R^{-1} (Q^T B)_{0:n} with [Q, R] = qr(W, 0), FP64.  Returns (X, R, ws)."""
    m, n = W.shape
    nrhs = B.shape[1] if B.dim() == 2 else 1
    if X is None:
        X = empty_colmajor(n, nrhs, torch.float64, W.device)
    if want_r and R is None:
        R = empty_colmajor(n, n, torch.float64, W.device)
    Wp, ldw = colmajor(W, "W")
    Bp, ldb = colmajor(B, "B")
    Xp, ldx = colmajor(X, "X")
    Rp, ldr = colmajor(R, "R") if R is not None else (None, n)
    need = workspace_size("qr_solve", n=n, nrhs=nrhs, k2=m)
    ws = workspace(need, W.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    _ok(_lib.ms_qr_solve(m, n, nrhs, Wp, ldw, Bp, ldb, Xp, ldx, Rp, ldr, wp, have,
                         _stream(stream)), "ms_qr_solve")
    return X, R, ws


def sketch_lstsq(A: torch.Tensor, B: torch.Tensor, h: torch.Tensor, s: torch.Tensor,
                 G: torch.Tensor, k: int, refine_steps: int = 0, mode: str = "auto",
                 X: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None,
                 tile_cols: int = 0, schedule: int = 0, y_terms: int = 0):
    """X = argmin || G C (B - A X) || (n x nrhs, FP64).  Returns (X, ws)."""
    d, n = A.shape
    if B.dim() == 1:
        B = B.unsqueeze(1)
    nrhs = B.shape[1]
    k2 = G.shape[0]
    a_dt, g_dt = _dt(A), _dt(G)
    if B.dtype != A.dtype:
        raise ValueError("B must have A's dtype")
    if X is None:
        X = empty_colmajor(n, nrhs, torch.float64, A.device)
    Ap, lda = colmajor(A, "A")
    Bp, ldb = colmajor(B, "B")
    Gp, ldg = colmajor(G, "G")
    Xp, ldx = colmajor(X, "X")
    need = workspace_size("lstsq", d=d, n=n, nrhs=nrhs, k=k, k2=k2, a_dtype=a_dt,
                          g_dtype=g_dt, mode=mode, refine_steps=refine_steps)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    o = _opts(mode, refine_steps, tile_cols, schedule, y_terms=y_terms)
    _ok(_lib.sketch_lstsq(d, n, nrhs, k, k2, a_dt, Ap, lda, Bp, ldb, _vec(h, torch.int32, "h"),
                          _vec(s, torch.int8, "s"), g_dt, Gp, ldg, Xp, ldx, ctypes.byref(o), wp,
                          have, _stream(stream)), "sketch_lstsq")
    return X, ws


def sketch_lstsq_noalloc(A: torch.Tensor, B: torch.Tensor, h: torch.Tensor, s: torch.Tensor,
                         G: torch.Tensor, k: int, X: torch.Tensor, status: torch.Tensor | None = None,
                         refine_steps: int = 0, mode: str = "auto", stream=None,
                         y_terms: int = 0):
    """sketch_lstsq with the library's static per-device scratch array instead
    of a workspace: the caller passes the inputs and the outputs X (n x nrhs,
    FP64, column-major) and optionally ``status`` (a 1-element int32 device
    tensor receiving the device-side status).  Allocates nothing.  Returns X."""
    d, n = A.shape
    if B.dim() == 1:
        B = B.unsqueeze(1)
    nrhs = B.shape[1]
    k2 = G.shape[0]
    a_dt, g_dt = _dt(A), _dt(G)
    if B.dtype != A.dtype:
        raise ValueError("B must have A's dtype")
    Ap, lda = colmajor(A, "A")
    Bp, ldb = colmajor(B, "B")
    Gp, ldg = colmajor(G, "G")
    Xp, ldx = colmajor(X, "X")
    Xs = X if X.dim() == 2 else X.unsqueeze(1)
    if X.dtype != torch.float64 or tuple(Xs.shape) != (n, nrhs):
        raise ValueError("X must be an n x nrhs FP64 tensor")
    sp = None
    if status is not None:
        sp = _vec(status.view(-1), torch.int32, "status")
    o = _opts(mode, refine_steps, y_terms=y_terms)
    _ok(_lib.sketch_lstsq_noalloc(d, n, nrhs, k, k2, a_dt, Ap, lda, Bp, ldb,
                                  _vec(h, torch.int32, "h"), _vec(s, torch.int8, "s"), g_dt, Gp,
                                  ldg, Xp, ldx, sp, ctypes.byref(o), _stream(stream)),
        "sketch_lstsq_noalloc")
    return X


def rand_cholqr_lstsq(A: torch.Tensor, B: torch.Tensor, h: torch.Tensor, s: torch.Tensor,
                      G: torch.Tensor, k: int, mode: str = "auto", X: torch.Tensor | None = None,
                      R: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None,
                      y_terms: int = 0):
    """X = argmin ||B - A X|| by rand_cholQR least squares with the multisketch
    G C as the sketch operator (n x nrhs, FP64; the least-squares optimum, no
    sketch distortion).  R (optional, n x n FP64) receives the R factor of A.
    Returns (X, R, ws)."""
    d, n = A.shape
    if B.dim() == 1:
        B = B.unsqueeze(1)
    nrhs = B.shape[1]
    k2 = G.shape[0]
    a_dt, g_dt = _dt(A), _dt(G)
    if B.dtype != A.dtype:
        raise ValueError("B must have A's dtype")
    if X is None:
        X = empty_colmajor(n, nrhs, torch.float64, A.device)
    Ap, lda = colmajor(A, "A")
    Bp, ldb = colmajor(B, "B")
    Gp, ldg = colmajor(G, "G")
    Xp, ldx = colmajor(X, "X")
    Rp, ldr = colmajor(R, "R") if R is not None else (None, n)
    need = workspace_size("rand_cholqr", d=d, n=n, nrhs=nrhs, k=k, k2=k2, a_dtype=a_dt,
                          g_dtype=g_dt, mode=mode)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    o = _opts(mode, 0, y_terms=y_terms)
    _ok(_lib.rand_cholqr_lstsq(d, n, nrhs, k, k2, a_dt, Ap, lda, Bp, ldb, _vec(h, torch.int32, "h"),
                               _vec(s, torch.int8, "s"), g_dt, Gp, ldg, Xp, ldx, Rp, ldr,
                               ctypes.byref(o), wp, have, _stream(stream)), "rand_cholqr_lstsq")
    return X, R, ws


def normal_equations_lstsq(A: torch.Tensor, B: torch.Tensor, X: torch.Tensor | None = None,
                           R: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                           stream=None):
    """X = argmin ||B - A X|| by the normal equations: [A | B]^T [A | B] in
    FP64 in one pass, R = chol(A^T A), R^T y = A^T B, X = R^{-1} y (n x nrhs,
    FP64).  R (optional, n x n FP64) receives the Cholesky factor.
    Returns (X, R, ws)."""
    d, n = A.shape
    if B.dim() == 1:
        B = B.unsqueeze(1)
    nrhs = B.shape[1]
    a_dt = _dt(A)
    if B.dtype != A.dtype:
        raise ValueError("B must have A's dtype")
    if X is None:
        X = empty_colmajor(n, nrhs, torch.float64, A.device)
    Ap, lda = colmajor(A, "A")
    Bp, ldb = colmajor(B, "B")
    Xp, ldx = colmajor(X, "X")
    Rp, ldr = colmajor(R, "R") if R is not None else (None, n)
    need = workspace_size("normal_equations", d=d, n=n, nrhs=nrhs, a_dtype=a_dt)
    ws = workspace(need, A.device) if ws is None else ws
    wp, have = _ws_ptr(ws, need)
    _ok(_lib.normal_equations_lstsq(d, n, nrhs, a_dt, Ap, lda, Bp, ldb, Xp, ldx, Rp, ldr, None,
                                    wp, have, _stream(stream)), "normal_equations_lstsq")
    return X, R, ws


# --------------------------------------------------------------------------
# Batched sketch-and-solve
# --------------------------------------------------------------------------

def _describe(prob: dict) -> MsProblem:
    """ms_problem of a dict with tensors A, B, h, s, G, X and the int k."""
    A, B, G, X = prob["A"], prob["B"], prob["G"], prob["X"]
    if B.dim() == 1:
        B = B.unsqueeze(1)
    Ap, lda = colmajor(A, "A")
    Bp, ldb = colmajor(B, "B")
    Gp, ldg = colmajor(G, "G")
    Xp, ldx = colmajor(X, "X")
    return MsProblem(A.shape[0], A.shape[1], B.shape[1], int(prob["k"]), G.shape[0],
                     Ap, lda, Bp, ldb, _vec(prob["h"], torch.int32, "h"),
                     _vec(prob["s"], torch.int8, "s"), Gp, ldg, Xp, ldx)


def _host_array(problems):
    """ms_problem array of problem dicts, or of (d, n, nrhs, k, k2) shape
    tuples (capacity sets only: the host-side descriptors that size the
    workspace and the launch shapes; their pointers are placeholders that no
    kernel reads -- the kernels read the device descriptors of the problems
    being solved)."""
    arr = (MsProblem * len(problems))()
    for i, pr in enumerate(problems):
        if isinstance(pr, tuple):
            d, n, nrhs, k, k2 = (int(v) for v in pr)
            ph = 256
            arr[i] = MsProblem(d, n, nrhs, k, k2, ph, d, ph, d, ph, ph, ph, k2, ph, n)
        else:
            arr[i] = _describe(pr)
    return arr


def batch_workspace_size(problems, a_dtype: int, g_dtype: int, rows_log2: int = 0,
                         kchunk_log2: int = 0, refine_steps: int = 0, y_terms: int = 0) -> int:
    arr = _host_array(problems)
    o = _opts("auto", refine_steps, 0, 0, rows_log2, kchunk_log2, y_terms)
    sz = _lib.ms_batch_workspace_size(len(problems), arr, a_dtype, g_dtype, ctypes.byref(o))
    if sz == 0:
        raise MsketchError(MS_ERR_ARG, "ms_batch_workspace_size")
    return sz


def batch_status(ws: torch.Tensor, count: int, stream=None):
    """(batch status, per-problem status list) of the last batched call on ws."""
    out = (ctypes.c_int32 * count)()
    p = (ws.data_ptr() + 255) // 256 * 256
    st = _lib.ms_batch_status(ctypes.c_void_p(p), count, out, _stream(stream))
    return st, list(out)


class BatchRunner:
    """A batched multisketch sketch-and-solve with its workspace and device
    descriptors, reusable across calls and capturable in a HIP graph.

    ``problems``: list of dicts with device tensors A (d x n), B (d x nrhs),
    h (int32, d), s (int8, d), G (k2 x k), X (n x nrhs, FP64) and int k.
    ``capacity``: problems that bound later ones (same count; the later
    sets' totals of sketch, partial, factor and residual sizes no larger);
    problem dicts or (d, n, nrhs, k, k2) tuples; defaults to ``problems``.
    ``refine_steps``: FP64-residual refinement steps (each problem then needs
    nrhs <= 8).  ``deterministic``: the CountSketch folds every bucket in
    ascending row order, so each problem's X does not depend on the rest of
    the batch (bit for bit).  ``refine_tol_log2`` (x > 0): a problem stops
    refining once a step's correction is at most 2^-x of its X (Frobenius).
    """

    def __init__(self, problems, capacity=None, rows_log2: int = 0, kchunk_log2: int = 0,
                 refine_steps: int = 0, y_terms: int = 0, deterministic: bool = False,
                 refine_tol_log2: int = 0):
        if not problems:
            raise ValueError("empty batch")
        self.count = len(problems)
        self.a_dtype = _dt(problems[0]["A"])
        self.g_dtype = _dt(problems[0]["G"])
        self.opts = _opts("sorted" if deterministic else "auto", refine_steps, 0, 0, rows_log2,
                          kchunk_log2, y_terms, refine_tol_log2)
        cap = capacity if capacity is not None else problems
        cap_arr = _host_array(cap)
        need = _lib.ms_batch_workspace_size(self.count, cap_arr, self.a_dtype, self.g_dtype,
                                            ctypes.byref(self.opts))
        if need == 0:
            raise MsketchError(MS_ERR_ARG, "ms_batch_workspace_size")
        dev = problems[0]["A"].device
        self.ws = workspace(need, dev)
        self.ws_ptr, self.ws_bytes = _ws_ptr(self.ws, need)
        self.cap_host = cap_arr          # launch shapes come from the capacity set
        nbytes = ctypes.sizeof(MsProblem) * self.count
        # staging buffers of the descriptor copies, used in turn: a buffer is
        # rewritten only once the copy that last read it has run (its event),
        # so set_problems may be called again before earlier work has ended
        self._stage = [torch.empty(nbytes, dtype=torch.uint8).pin_memory()
                       for _ in range(self.STAGING)]
        self._stage_done = [None] * self.STAGING
        self._next_stage = 0
        self.desc_dev = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.graph = None
        self.set_problems(problems)

    STAGING = 3

    def set_problems(self, problems, stream=None):
        """Rewrite the device descriptors (a stream-ordered copy: launches or
        replays enqueued before it on the stream use the earlier problems)."""
        if len(problems) != self.count:
            raise ValueError("a runner keeps its problem count")
        arr = _host_array(problems)
        i = self._next_stage
        self._next_stage = (i + 1) % self.STAGING
        if self._stage_done[i] is not None:
            self._stage_done[i].synchronize()
        ctypes.memmove(self._stage[i].data_ptr(), arr, ctypes.sizeof(arr))
        s = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            self.desc_dev.copy_(self._stage[i], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self._stage_done[i] = ev
        self.problems = problems

    def launch(self, stream=None):
        _ok(_lib.sketch_lstsq_batched(self.count, self.cap_host,
                                      ctypes.c_void_p(self.desc_dev.data_ptr()), self.a_dtype,
                                      self.g_dtype, ctypes.byref(self.opts),
                                      ctypes.c_void_p(self.ws_ptr), self.ws_bytes,
                                      _stream(stream)), "sketch_lstsq_batched")

    def capture(self):
        """Capture one launch sequence in a graph (torch.cuda.CUDAGraph)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.launch(s)          # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch(torch.cuda.current_stream())
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def status(self, stream=None):
        return batch_status(self.ws, self.count, stream)


def sketch_lstsq_batched(problems, rows_log2: int = 0, kchunk_log2: int = 0,
                         refine_steps: int = 0, stream=None, y_terms: int = 0,
                         deterministic: bool = False, refine_tol_log2: int = 0):
    """Solve a list of problems (dicts as for BatchRunner) in one batched call;
    returns the runner (its problems' X tensors hold the solutions)."""
    r = BatchRunner(problems, rows_log2=rows_log2, kchunk_log2=kchunk_log2,
                    refine_steps=refine_steps, y_terms=y_terms, deterministic=deterministic,
                    refine_tol_log2=refine_tol_log2)
    r.launch(stream)
    return r
