"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point ``include/msketch.h`` declares, sizes workspaces, and
rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msketch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s+\**([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def ms():
    import paper_2508_14209_amd as ms
    return ms


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["countsketch_apply", "multisketch_apply", "sketch_lstsq", "ms_bucket_plan",
              "ms_gaussian_apply", "ms_qr_solve", "ms_workspace_size", "ms_check_status",
              "ms_status_string"]:
        assert n in names, n


def test_library_exports_every_declared_symbol(ms):
    lib = ctypes.CDLL(ms.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_sizes(ms):
    for op, kw in [("bucket_plan", dict(d=1000, k=64)),
                   ("countsketch", dict(d=1000, n=3, k=64)),
                   ("countsketch", dict(d=1000, n=3, k=64, mode="sorted")),
                   ("gaussian", dict(n=9, k=128, k2=16)),
                   ("multisketch", dict(d=1000, n=8, k=128, k2=16)),
                   ("qr_solve", dict(n=64, nrhs=1, k2=128)),
                   ("lstsq", dict(d=4194304, n=64, nrhs=1, k=8192, k2=128)),
                   ("lstsq", dict(d=1 << 20, n=32, nrhs=4, k=2048, k2=64, a_dtype=1, g_dtype=2,
                                  refine_steps=3))]:
        sz = ms.workspace_size(op, **kw)
        assert sz >= 256 and sz % 256 == 0, (op, kw, sz)
    # the sorted plan needs more room than the packed codes
    assert ms.workspace_size("countsketch", d=10 ** 6, n=3, k=64, mode="sorted") > \
        ms.workspace_size("countsketch", d=10 ** 6, n=3, k=64, mode="lds")
    # refinement buffers are only carved when asked for
    a = ms.workspace_size("lstsq", d=1 << 20, n=32, nrhs=4, k=2048, k2=64, a_dtype=1, g_dtype=2)
    b = ms.workspace_size("lstsq", d=1 << 20, n=32, nrhs=4, k=2048, k2=64, a_dtype=1, g_dtype=2,
                          refine_steps=1)
    assert b > a + (1 << 20) * 4 * 8


def test_invalid_arguments_rejected_on_host(ms):
    lib = ms._lib
    ws = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    o = ms.MsOpts(0, 0, 0, 0, 0, 0, 0, 0)
    P = ctypes.c_void_p(0x2000)
    # negative sizes, k < 1, lda < d, unknown dtype, unknown mode, null workspace
    assert lib.countsketch_apply(-1, 1, 4, 0, P, 1, P, P, P, 4, ctypes.byref(o), ws, 1 << 20, None) == ms.MS_ERR_ARG
    assert lib.countsketch_apply(10, 1, 0, 0, P, 10, P, P, P, 4, ctypes.byref(o), ws, 1 << 20, None) == ms.MS_ERR_ARG
    assert lib.countsketch_apply(10, 1, 4, 0, P, 9, P, P, P, 4, ctypes.byref(o), ws, 1 << 20, None) == ms.MS_ERR_ARG
    assert lib.countsketch_apply(10, 1, 4, 7, P, 10, P, P, P, 4, ctypes.byref(o), ws, 1 << 20, None) == ms.MS_ERR_ARG
    assert lib.countsketch_apply(10, 1, 4, 0, P, 10, P, P, P, 4, ctypes.byref(o), None, 1 << 20, None) == ms.MS_ERR_ARG
    bad = ms.MsOpts(9, 0, 0, 0, 0, 0, 0, 0)
    assert lib.countsketch_apply(10, 1, 4, 0, P, 10, P, P, P, 4, ctypes.byref(bad), ws, 1 << 20, None) == ms.MS_ERR_ARG
    # workspace too small
    assert lib.countsketch_apply(10, 1, 4, 0, P, 10, P, P, P, 4, ctypes.byref(o), ws, 16, None) == ms.MS_ERR_NOMEM
    # dtype combinations the Gaussian stage does not support
    assert lib.ms_gaussian_apply(8, 2, 4, 0, P, 4, 1, P, 8, P, 4, ws, 1 << 20, None) == ms.MS_ERR_ARG
    assert lib.ms_gaussian_apply(8, 2, 4, 2, P, 4, 0, P, 8, P, 4, ws, 1 << 20, None) == ms.MS_ERR_ARG
    # k2 < n for least squares; refinement with too many right-hand sides
    assert lib.sketch_lstsq(100, 8, 1, 32, 4, 0, P, 100, P, 100, P, P, 0, P, 4, P, 8,
                            ctypes.byref(o), ws, 1 << 30, None) == ms.MS_ERR_ARG
    r = ms.MsOpts(0, 2, 0, 0, 0, 0, 0, 0)
    assert lib.sketch_lstsq(100, 8, 9, 32, 16, 1, P, 100, P, 100, P, P, 1, P, 16, P, 8,
                            ctypes.byref(r), ws, 1 << 30, None) == ms.MS_ERR_UNSUPPORTED
    # QR: m < n
    assert lib.ms_qr_solve(4, 8, 1, P, 4, P, 4, P, 8, None, 8, ws, 1 << 20, None) == ms.MS_ERR_ARG
    assert lib.ms_check_status(None, None) == ms.MS_ERR_ARG
    assert lib.ms_workspace_size(99, 1, 1, 1, 1, 1, 0, 0, None) == 0


def test_status_strings(ms):
    for code in range(7):
        assert ms._lib.ms_status_string(code).decode().startswith("MS_")


def test_struct_layouts_match_binding(ms, tmp_path):
    # the C compiler's view of the ABI structs equals the ctypes mirrors
    src = tmp_path / "sz.c"
    src.write_text('#include "msketch.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(ms_opts), sizeof(ms_problem),'
                   ' offsetof(ms_problem, X), offsetof(ms_opts, batch_kchunk_log2));return 0;}\n')
    exe = tmp_path / "sz"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert int(out[0]) == ctypes.sizeof(ms.MsOpts)
    assert int(out[1]) == ctypes.sizeof(ms.MsProblem)
    assert int(out[2]) == ms.MsProblem.X.offset
    assert int(out[3]) == ms.MsOpts.batch_kchunk_log2.offset


def test_batch_workspace_size_host_only(ms):
    import torch
    # descriptors are only inspected on the host here: fake device pointers
    P = ms.MsProblem(1000, 8, 2, 128, 16, 0x10000, 1000, 0x20000, 1000, 0x30000, 0x40000,
                     0x50000, 16, 0x60000, 8)
    arr = (ms.MsProblem * 2)(P, P)
    o = ms.MsOpts(0, 0, 0, 0, 0, 0, 0, 0)
    sz = ms._lib.ms_batch_workspace_size(2, arr, 1, 1, ctypes.byref(o))
    assert sz >= 256 and sz % 256 == 0
    # k2 above the batched limit, bad tuning: refused
    Pbig = ms.MsProblem(1000, 8, 2, 128, 512, 0x10000, 1000, 0x20000, 1000, 0x30000, 0x40000,
                        0x50000, 512, 0x60000, 8)
    assert ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(Pbig), 1, 1, ctypes.byref(o)) == 0
    # refinement adds the QR factors, the FP64 residual (d x nrhs), its sketch
    # (k x nrhs) and the residual's Gaussian-stage partials, each 256-aligned
    # (without refinement each of the four areas is one empty 256-byte block)
    r = ms.MsOpts(0, 1, 0, 0, 0, 0, 0, 0)
    one = ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(P), 1, 1, ctypes.byref(o))
    one_r = ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(P), 1, 1, ctypes.byref(r))
    al = lambda x: (x + 255) // 256 * 256
    assert one_r - one == (al((16 * 8 + 8) * 8) + al(1000 * 2 * 8) + al(128 * 2 * 8)
                           + al(1 * 16 * 2 * 8) - 4 * 256)
    # refinement needs nrhs <= 8; at most 64 steps
    P9 = ms.MsProblem(1000, 8, 9, 128, 16, 0x10000, 1000, 0x20000, 1000, 0x30000, 0x40000,
                      0x50000, 16, 0x60000, 8)
    assert ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(P9), 1, 1, ctypes.byref(o)) > 0
    assert ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(P9), 1, 1, ctypes.byref(r)) == 0
    assert ms._lib.sketch_lstsq_batched(1, (ms.MsProblem * 1)(P9), (ms.MsProblem * 1)(P9), 1, 1,
                                        ctypes.byref(r), ctypes.c_void_p(0x1000), 1 << 30,
                                        None) == ms.MS_ERR_UNSUPPORTED
    r65 = ms.MsOpts(0, 65, 0, 0, 0, 0, 0, 0)
    assert ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(P), 1, 1, ctypes.byref(r65)) == 0
    bad = ms.MsOpts(0, 0, 0, 0, 30, 0, 0, 0)
    assert ms._lib.ms_batch_workspace_size(1, (ms.MsProblem * 1)(P), 1, 1, ctypes.byref(bad)) == 0
    assert ms._lib.sketch_lstsq_batched(0, arr, arr, 1, 1, None, ctypes.c_void_p(0x1000), 1 << 30,
                                        None) == ms.MS_ERR_ARG


def test_workspace_sizes_of_the_later_rows(ms):
    # rand_cholQR, normal equations, hash-generated CountSketch, SRHT, Count + SRHT
    for op, kw in [("rand_cholqr", dict(d=4194304, n=64, nrhs=1, k=8192, k2=128)),
                   ("normal_equations", dict(d=4194304, n=64, nrhs=1)),
                   ("countsketch_hashed", dict(d=1 << 24, n=8, k=128, a_dtype=1)),
                   ("srht", dict(d=4194304, n=64, k=128)),
                   ("srht", dict(d=5000, n=3, k=16)),
                   ("count_srht_lstsq", dict(d=4194304, n=64, nrhs=1, k=8192, k2=128))]:
        sz = ms.workspace_size(op, **kw)
        assert sz >= 256 and sz % 256 == 0, (op, kw, sz)
    # the SRHT keeps per-block partials only past one 8192-row block:
    # 512 blocks x 64 columns x 128 rows x 8 bytes for 4,194,304 rows
    assert ms.workspace_size("srht", d=4194304, n=64, k=128) >= 512 * 64 * 128 * 8
    assert ms.workspace_size("srht", d=8192, n=64, k=128) < 4096


def test_later_rows_reject_invalid_arguments_on_host(ms):
    lib = ms._lib
    ws = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    P = ctypes.c_void_p(0x2000)
    o = ms.MsOpts(0, 0, 0, 0, 0, 0, 0, 0)
    refine = ms.MsOpts(0, 1, 0, 0, 0, 0, 0, 0)
    sorted_ = ms.MsOpts(3, 0, 0, 0, 0, 0, 0, 0)
    big = 1 << 30
    # normal equations: n > 256, nrhs > 16 unsupported; nrhs = 0 invalid
    assert lib.normal_equations_lstsq(300, 257, 1, 0, P, 300, P, 300, P, 257, None, 257, None, ws,
                                      big, None) == ms.MS_ERR_UNSUPPORTED
    assert lib.normal_equations_lstsq(100, 8, 17, 0, P, 100, P, 100, P, 8, None, 8, None, ws,
                                      big, None) == ms.MS_ERR_UNSUPPORTED
    assert lib.normal_equations_lstsq(100, 8, 0, 0, P, 100, P, 100, P, 8, None, 8, None, ws,
                                      big, None) == ms.MS_ERR_ARG
    # rand_cholQR: no refinement steps; k2 >= n
    assert lib.rand_cholqr_lstsq(100, 8, 1, 128, 16, 0, P, 100, P, 100, P, P, 0, P, 16, P, 8,
                                 None, 8, ctypes.byref(refine), ws, big, None) == ms.MS_ERR_ARG
    assert lib.rand_cholqr_lstsq(100, 8, 1, 128, 4, 0, P, 100, P, 100, P, P, 0, P, 4, P, 8,
                                 None, 8, ctypes.byref(o), ws, big, None) == ms.MS_ERR_ARG
    # hash-generated CountSketch: LDS schedule only; k in [1, 2^31 - 2]
    assert lib.countsketch_hashed(100, 2, 16, 7, 0, P, 100, P, 16, ctypes.byref(sorted_), ws, big,
                                  None) == ms.MS_ERR_UNSUPPORTED
    assert lib.countsketch_hashed(100, 2, 0, 7, 0, P, 100, P, 16, ctypes.byref(o), ws, big,
                                  None) == ms.MS_ERR_ARG
    assert lib.ms_hash_sketch(10, 0, 1, P, P, None) == ms.MS_ERR_ARG
    assert lib.ms_hash_sketch(10, (1 << 31) - 1, 1, P, P, None) == ms.MS_ERR_ARG
    assert lib.ms_hash_sketch(10, 16, 1, None, P, None) == ms.MS_ERR_ARG
    # SRHT: m >= 1, k >= 1, at most 65535 columns, FP64 or FP32 data
    assert lib.srht_apply(0, 2, 4, 0, P, 1, P, P, P, 4, ws, big, None) == ms.MS_ERR_ARG
    assert lib.srht_apply(100, 2, 0, 0, P, 100, P, P, P, 4, ws, big, None) == ms.MS_ERR_ARG
    assert lib.srht_apply(100, 70000, 4, 0, P, 100, P, P, P, 4, ws, big, None) == ms.MS_ERR_ARG
    assert lib.srht_apply(100, 2, 4, 2, P, 100, P, P, P, 4, ws, big, None) == ms.MS_ERR_ARG
    # Count + SRHT least squares: k2 >= n, no refinement
    assert lib.count_srht_lstsq(100, 8, 1, 128, 4, 0, P, 100, P, 100, P, P, P, P, P, 8,
                                ctypes.byref(o), ws, big, None) == ms.MS_ERR_ARG
    assert lib.count_srht_lstsq(100, 8, 1, 128, 16, 0, P, 100, P, 100, P, P, P, P, P, 8,
                                ctypes.byref(refine), ws, big, None) == ms.MS_ERR_ARG


def test_request_generator_rejects_invalid_arguments_on_host(ms):
    lib = ms._lib
    P = ctypes.c_void_p(0x2000)  # never dereferenced: every call below fails validation first
    F32, BF16, F16 = ms.MS_F32, ms.MS_BF16, ms.MS_F16

    def gen(d=100, n=8, nrhs=2, kappa=10.0, k=128, k2=16, gdt=F32, A=P, lda=100, B=P, ldb=100,
            h=P, s=P, G=P):
        return lib.ms_gen_lstsq_request(1, d, n, nrhs, kappa, 1e-6, k, k2, gdt, A, lda, B, ldb, P,
                                        h, s, G, None)
    assert gen(n=0) == ms.MS_ERR_ARG
    assert gen(n=129) == ms.MS_ERR_ARG            # rows are formed in registers: n <= 128
    assert gen(nrhs=0) == ms.MS_ERR_ARG
    assert gen(nrhs=9) == ms.MS_ERR_ARG
    assert gen(d=0) == ms.MS_ERR_ARG
    assert gen(kappa=0.5) == ms.MS_ERR_ARG
    assert gen(kappa=float("inf")) == ms.MS_ERR_ARG
    assert gen(kappa=float("nan")) == ms.MS_ERR_ARG
    assert gen(k=0) == ms.MS_ERR_ARG
    assert gen(k2=(1 << 31) - 1) == ms.MS_ERR_ARG
    assert gen(lda=99) == ms.MS_ERR_ARG
    assert gen(ldb=99) == ms.MS_ERR_ARG
    assert gen(A=None) == ms.MS_ERR_ARG            # B is formed from A's rows
    assert gen(h=None) == ms.MS_ERR_ARG            # h and s come together
    assert gen(gdt=F16) == ms.MS_ERR_ARG
