"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/oracle.c``, plants one plausible mistake (a dropped
sign, a wrong index, a transposed operand, a reversed fold, a broken sign
convention, ...), builds the mutant on the CPU and runs the oracle pin suite
against it in a subprocess: the suite has to fail.  This checks that the pins
are strong enough to tell a wrong oracle from the right one.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, original text, mutated text, which occurrence (0-based) to change)
MUTANTS = [
    ("cs64_sign_dropped", "Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);",
     "Y[m + c * ldy] = Y[m + c * ldy] + a;", 0),
    ("cs32_sign_flipped", "Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);",
     "Y[m + c * ldy] = Y[m + c * ldy] + (s[i] < 0 ? a : -a);", 1),
    ("cs64_fold_reversed", "for (int64_t i = 0; i < d; ++i) {\n    const int64_t m = h[i];",
     "for (int64_t i = d - 1; i >= 0; --i) {\n    const int64_t m = h[i];", 0),
    # FP32 data folded in FP64: a float fold and a flipped sign
    ("cs32acc64_float_fold", "const double a = (double)A[i + c * lda];\n      Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);",
     "const float a = A[i + c * lda];\n      Y[m + c * ldy] = (float)((float)Y[m + c * ldy] + (s[i] > 0 ? a : -a));", 0),
    ("cs32acc64_sign_flipped", "Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);",
     "Y[m + c * ldy] = Y[m + c * ldy] + (s[i] < 0 ? a : -a);", 2),
    ("cols_fold_sign_dropped", "j->Y[m + c * j->ldy] = j->Y[m + c * j->ldy] + (j->s[i] > 0 ? a : -a);",
     "j->Y[m + c * j->ldy] = j->Y[m + c * j->ldy] + a;", 0),
    ("cols_split_skips_last_column", "or_cs_cols_job j = {d, k, n * t / nthreads, n * (t + 1) / nthreads,",
     "or_cs_cols_job j = {d, k, n * t / nthreads, n * (t + 1) / nthreads - (t + 1 == nthreads),", 0),
    ("cs64_bucket_shift", "const int64_t m = h[i];", "const int64_t m = (h[i] + 1) % k;", 0),
    ("cs64_init_neg_zero", "for (int64_t m = 0; m < k; ++m) Y[m + c * ldy] = +0.0;",
     "for (int64_t m = 0; m < k; ++m) Y[m + c * ldy] = -0.0;", 0),
    ("hist_skip_first_row", "for (int64_t i = 0; i < d; ++i) cnt[h[i]] += 1;",
     "for (int64_t i = 1; i < d; ++i) cnt[h[i]] += 1;", 0),
    ("plan_unstable", "for (int64_t i = 0; i < d; ++i) perm[cnt[h[i]]++] = i;",
     "for (int64_t i = d - 1; i >= 0; --i) perm[cnt[h[i]]++] = i;", 0),
    ("gemm_transposed_G", "acc = acc + G[p + m * ldg] * Y[m + c * ldy];",
     "acc = acc + G[m + p * ldg] * Y[m + c * ldy];", 0),
    ("gemm_dropped_term", "for (int64_t m = 0; m < K; ++m)\n        acc = acc + G",
     "for (int64_t m = 1; m < K; ++m)\n        acc = acc + G", 0),
    ("qr_sign_convention", "const double beta = alpha >= 0.0 ? -norm : norm;",
     "const double beta = alpha >= 0.0 ? norm : -norm;", 0),
    ("qr_update_without_tau", "      w = w * tau[j];\n      cc[j] = cc[j] - w;",
     "      cc[j] = cc[j] - w;", 0),
    ("qt_skips_leading_one", "double w = bc[j];", "double w = 0.0;", 0),
    ("trsv_transposed", "acc = acc - R[i + j * ldr] * x[j];", "acc = acc - R[j + i * ldr] * x[j];", 0),
    ("ne_forward_wrong_index", "acc = acc - Gm[t + i * n] * x[t];", "acc = acc - Gm[i + t * n] * x[t];", 0),
    ("composite_rhs_offset", "st = or_countsketch_f64(d, nrhs, k, B, ldb, h, s, Y + n * k, k);",
     "st = or_countsketch_f64(d, nrhs, k, B, ldb, h, s, Y + (n - 1) * k, k);", 0),
    # the FP64-fold FP32 sketch of the FP32 least-squares path
    ("acc64_rhs_offset", "st = or_countsketch_f32_acc64(d, nrhs, k, B, ldb, h, s, Yd + n * k, k);",
     "st = or_countsketch_f32_acc64(d, nrhs, k, B, ldb, h, s, Yd + (n - 1) * k, k);", 0),
    ("acc64_rounds_to_bf16", "for (int64_t t = 0; t < k * nc; ++t) Y[t] = (float)Yd[t];",
     "for (int64_t t = 0; t < k * nc; ++t) Y[t] = or_round_bf16((float)Yd[t]);", 0),
    ("bf16_ties_away", "u = u + 0x7fffu + lsb;", "u = u + 0x8000u + 0 * lsb;", 0),
    # rand_cholQR least squares (Alg. 5)
    ("rcq_no_cholesky_correction", "for (int64_t t = i; t <= j; ++t) acc = acc + Gm[i + t * n] * W[t + j * m];",
     "acc = W[i + j * m];", 0),
    ("rcq_r1_not_transposed", "for (int64_t t = 0; t < i; ++t) acc = acc - Gm[t + i * n] * y[t];",
     "for (int64_t t = 0; t < i; ++t) acc = acc - Gm[i + t * n] * y[t];", 0),
    ("rcq_q0_times_r0", "for (int64_t l = 0; l < j; ++l) acc = acc - q[l] * W[l + j * m];\n      q[j] = acc / W[j + j * m];",
     "for (int64_t l = 0; l < j; ++l) acc = acc - q[l] * W[l + j * m];\n      q[j] = acc * W[j + j * m];", 0),
    ("rcq_rhs_skips_first_row", "for (int64_t p = 0; p < n; ++p) z[p + c * n] = z[p + c * n] + q[p] * B[i + c * ldb];",
     "if (i > 0) for (int64_t p = 0; p < n; ++p) z[p + c * n] = z[p + c * n] + q[p] * B[i + c * ldb];", 0),
    ("mix64_wrong_shift", "z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);",
     "z = (z ^ (z >> 31)) * UINT64_C(0xBF58476D1CE4E5B9);", 0),
    ("hash_bucket_low_bits", "h[i] = (int32_t)(((u >> 32) * (uint64_t)k) >> 32);",
     "h[i] = (int32_t)(((u & 0xffffffffu) * (uint64_t)k) >> 32);", 0),
    ("srht_sign_from_or", "acc = or_parity64((uint64_t)r[j] & (uint64_t)i) ? acc - v : acc + v;",
     "acc = or_parity64((uint64_t)r[j] | (uint64_t)i) ? acc - v : acc + v;", 0),
    ("srht_dsign_dropped", "const long double v = (long double)dsign[i] * (long double)X[i + c * ldx];",
     "const long double v = (long double)X[i + c * ldx];", 0),
    ("srht_scale_one_over_k", "const long double scale = 1.0L / sqrtl((long double)k);",
     "const long double scale = 1.0L / (long double)k;", 0),
    ("hash_row_off_by_one", "or_mix64(seed + (uint64_t)(i + 1) * UINT64_C(0x9E3779B97F4A7C15));",
     "or_mix64(seed + (uint64_t)i * UINT64_C(0x9E3779B97F4A7C15));", 0),
    # FP16 Gaussian-stage reference: rounding and the per-column scale
    ("f16_ties_away", "const double r = ldexp(nearbyint(ldexp(a, -q)), q);",
     "const double r = ldexp(round(ldexp(a, -q)), q);", 0),
    ("f16_no_subnormals", "if (q < -24) q = -24;", "if (q < -14) q = -14;", 0),
    ("f16_overflow_late", "r >= 65536.0 ? INFINITY", "r > 65536.0 ? INFINITY", 0),
    ("f16_colexp_off_by_one", "int e = E - 1 - 14;", "int e = E - 14;", 0),
    ("f16_scale_not_restored", "out[i + c * ldo] = ldexp((double)or_round_f16(y[i] * down), e);",
     "out[i + c * ldo] = (double)or_round_f16(y[i] * down);", 0),
]


def _mutate(src: str, old: str, new: str, occ: int) -> str:
    idx = -1
    for _ in range(occ + 1):
        idx = src.find(old, idx + 1)
        assert idx >= 0, "mutation anchor not found: %r" % old
    return src[:idx] + new + src[idx + len(old):]


def _run_mutant(args):
    name, old, new, occ, tmp = args
    src = open(SRC).read()
    mdir = os.path.join(tmp, name)
    os.makedirs(mdir)
    mc = os.path.join(mdir, "oracle.c")
    with open(mc, "w") as f:
        f.write(_mutate(src, old, new, occ))
    with open(os.path.join(mdir, "oracle.h"), "w") as f:
        f.write(open(os.path.join(ROOT, "oracle", "oracle.h")).read())
    lib = os.path.join(mdir, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                           "-fPIC", "-shared", mc, "-o", lib, "-lm"])
    env = dict(os.environ, MSKETCH_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_countsketch.py"),
                        os.path.join(ROOT, "tests", "test_oracle_solve.py"),
                        os.path.join(ROOT, "tests", "test_oracle_rcq.py"),
                        os.path.join(ROOT, "tests", "test_oracle_hash.py"),
                        os.path.join(ROOT, "tests", "test_oracle_srht.py"),
                        os.path.join(ROOT, "tests", "test_oracle_f16.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_every_planted_mistake_is_caught():
    src = open(SRC).read()
    for name, old, new, occ in MUTANTS:
        assert src.count(old) > occ, name
    with tempfile.TemporaryDirectory() as tmp:
        jobs = [(n, o, w, k, tmp) for (n, o, w, k) in MUTANTS]
        with ThreadPoolExecutor(max(1, min(6, (os.cpu_count() or 2) - 1))) as ex:
            results = list(ex.map(_run_mutant, jobs))
    survivors = [(n, out) for (n, rc, out) in results if rc == 0]
    assert not survivors, "mutants not caught by the oracle pins: %s" % survivors
    assert all(rc == 1 for (_, rc, _) in results), [(n, rc) for (n, rc, _) in results]
