/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the
 * CountSketch -> Gaussian multisketch -> sketch-and-solve least-squares path
 * of Higgins, Boman, Yamazaki, "A High Performance GPU CountSketch
 * Implementation and Its Application to Multisketching and Least Squares
 * Problems" (arXiv 2508.14209).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Conventions (readings of the paper, each listed in the design notes):
 *   - matrices are column-major with a leading dimension (LAPACK style);
 *   - the bucket map h is 0-based, h[i] in [0,k) (the paper numbers buckets
 *     1..k in Def. 3);
 *   - the sign s[i] is +1 or -1 (the paper's boolean "s_j ? A_j : -A_j" of
 *     Alg. 2 with true <=> +1);
 *   - every output is overwritten; accumulation starts from +0.0.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared (no FMA
 * contraction, IEEE round-to-nearest-even throughout).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* CountSketch (Def. 3; the row-bucket identity, Eq. (2); Alg. 2)            */
/* ------------------------------------------------------------------------ */

/*
 * Y = S*A where column i of S is s[i]*e_{h[i]} (Def. 3).  By Eq. (2) row m
 * of Y is the signed sum of the rows of A whose bucket is m.  The sum for each
 * bucket is folded in ascending row order starting from +0.0, in the output
 * precision; adding or subtracting a row is selected by the sign (Alg. 2), so
 * no multiply takes place.  Rows whose h is outside [0,k) or whose s is not
 * +-1 make the call return ORACLE_ERR_RANGE before anything is written.
 */
int or_countsketch_f64(int64_t d, int64_t n, int64_t k, const double *A,
                       int64_t lda, const int32_t *h, const int8_t *s,
                       double *Y, int64_t ldy) {
  for (int64_t i = 0; i < d; ++i)
    if (h[i] < 0 || h[i] >= k || (s[i] != 1 && s[i] != -1))
      return ORACLE_ERR_RANGE;
  for (int64_t c = 0; c < n; ++c)
    for (int64_t m = 0; m < k; ++m) Y[m + c * ldy] = +0.0;
  for (int64_t i = 0; i < d; ++i) {
    const int64_t m = h[i];
    for (int64_t c = 0; c < n; ++c) {
      const double a = A[i + c * lda];
      Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);
    }
  }
  return ORACLE_OK;
}

/* Same definition with FP32 data and FP32 accumulation. */
int or_countsketch_f32(int64_t d, int64_t n, int64_t k, const float *A,
                       int64_t lda, const int32_t *h, const int8_t *s,
                       float *Y, int64_t ldy) {
  for (int64_t i = 0; i < d; ++i)
    if (h[i] < 0 || h[i] >= k || (s[i] != 1 && s[i] != -1))
      return ORACLE_ERR_RANGE;
  for (int64_t c = 0; c < n; ++c)
    for (int64_t m = 0; m < k; ++m) Y[m + c * ldy] = +0.0f;
  for (int64_t i = 0; i < d; ++i) {
    const int64_t m = h[i];
    for (int64_t c = 0; c < n; ++c) {
      const float a = A[i + c * lda];
      Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);
    }
  }
  return ORACLE_OK;
}

/* Same definition for FP32 data promoted exactly to FP64 and folded in FP64
 * (the "plain FP64" reading of an FP32 matrix). */
int or_countsketch_f32_acc64(int64_t d, int64_t n, int64_t k, const float *A,
                             int64_t lda, const int32_t *h, const int8_t *s,
                             double *Y, int64_t ldy) {
  for (int64_t i = 0; i < d; ++i)
    if (h[i] < 0 || h[i] >= k || (s[i] != 1 && s[i] != -1))
      return ORACLE_ERR_RANGE;
  for (int64_t c = 0; c < n; ++c)
    for (int64_t m = 0; m < k; ++m) Y[m + c * ldy] = +0.0;
  for (int64_t i = 0; i < d; ++i) {
    const int64_t m = h[i];
    for (int64_t c = 0; c < n; ++c) {
      const double a = (double)A[i + c * lda];
      Y[m + c * ldy] = Y[m + c * ldy] + (s[i] > 0 ? a : -a);
    }
  }
  return ORACLE_OK;
}

/* The same FP64 fold on several host threads, split by column: each column
 * is folded by one thread in exactly the canonical order above (ascending
 * rows from +0.0), and columns do not interact, so the result is bit for bit
 * that of or_countsketch_f64.  Used to time the oracle on all host cores. */
typedef struct {
  int64_t d, k, c0, c1, lda, ldy;
  const double *A;
  const int32_t *h;
  const int8_t *s;
  double *Y;
} or_cs_cols_job;

static void *or_cs_cols_run(void *arg) {
  const or_cs_cols_job *j = (const or_cs_cols_job *)arg;
  for (int64_t c = j->c0; c < j->c1; ++c)
    for (int64_t m = 0; m < j->k; ++m) j->Y[m + c * j->ldy] = +0.0;
  for (int64_t i = 0; i < j->d; ++i) {
    const int64_t m = j->h[i];
    for (int64_t c = j->c0; c < j->c1; ++c) {
      const double a = j->A[i + c * j->lda];
      j->Y[m + c * j->ldy] = j->Y[m + c * j->ldy] + (j->s[i] > 0 ? a : -a);
    }
  }
  return NULL;
}

int or_countsketch_f64_cols(int64_t d, int64_t n, int64_t k, const double *A,
                            int64_t lda, const int32_t *h, const int8_t *s,
                            double *Y, int64_t ldy, int nthreads) {
  for (int64_t i = 0; i < d; ++i)
    if (h[i] < 0 || h[i] >= k || (s[i] != 1 && s[i] != -1))
      return ORACLE_ERR_RANGE;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n) nthreads = n > 0 ? (int)n : 1;
  pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
  int *live = (int *)calloc((size_t)nthreads, sizeof(int));
  or_cs_cols_job *jobs = (or_cs_cols_job *)malloc((size_t)nthreads * sizeof(or_cs_cols_job));
  if (!th || !live || !jobs) {
    free(th);
    free(live);
    free(jobs);
    return ORACLE_ERR_NOMEM;
  }
  for (int t = 0; t < nthreads; ++t) {
    or_cs_cols_job j = {d, k, n * t / nthreads, n * (t + 1) / nthreads, lda, ldy, A, h, s, Y};
    jobs[t] = j;
  }
  for (int t = 1; t < nthreads; ++t)
    live[t] = pthread_create(&th[t], NULL, or_cs_cols_run, &jobs[t]) == 0;
  or_cs_cols_run(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) {
    if (live[t])
      pthread_join(th[t], NULL);
    else
      or_cs_cols_run(&jobs[t]); /* no thread could start: fold those columns here */
  }
  free(th);
  free(live);
  free(jobs);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Sketch plan: bucket histogram, exclusive scan, stable counting sort.      */
/* The paper only notes that the parallel fold of Alg. 2 needs atomics; the  */
/* plan groups the rows of each bucket in ascending row order, which is the  */
/* order the canonical fold above visits them in.                            */
/* ------------------------------------------------------------------------ */

int or_bucket_hist(int64_t d, int64_t k, const int32_t *h, int64_t *cnt) {
  for (int64_t i = 0; i < d; ++i)
    if (h[i] < 0 || h[i] >= k) return ORACLE_ERR_RANGE;
  for (int64_t m = 0; m < k; ++m) cnt[m] = 0;
  for (int64_t i = 0; i < d; ++i) cnt[h[i]] += 1;
  return ORACLE_OK;
}

/* off has k+1 entries: off[m] = number of rows in buckets < m; perm lists the
 * rows of bucket 0, then bucket 1, ..., each group in ascending row order. */
int or_bucket_plan(int64_t d, int64_t k, const int32_t *h, int64_t *off,
                   int64_t *perm) {
  int64_t *cnt = (int64_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int64_t));
  if (!cnt) return ORACLE_ERR_NOMEM;
  int st = or_bucket_hist(d, k, h, cnt);
  if (st != ORACLE_OK) {
    free(cnt);
    return st;
  }
  off[0] = 0;
  for (int64_t m = 0; m < k; ++m) off[m + 1] = off[m] + cnt[m];
  /* cnt now serves as the running cursor of each bucket */
  for (int64_t m = 0; m < k; ++m) cnt[m] = off[m];
  for (int64_t i = 0; i < d; ++i) perm[cnt[h[i]]++] = i;
  free(cnt);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Gaussian stage (Sec. 1, multisketch S2(S1 x); Table 1)                    */
/* ------------------------------------------------------------------------ */

/* Z = G*Y, M x N = (M x K)(K x N), every dot product folded in ascending
 * inner index from +0.0 in FP64.  Inputs are FP64 arrays; a caller holding
 * FP32 or BF16 values passes their exact FP64 images. */
void or_gemm_f64(int64_t M, int64_t N, int64_t K, const double *G, int64_t ldg,
                 const double *Y, int64_t ldy, double *Z, int64_t ldz) {
  for (int64_t c = 0; c < N; ++c)
    for (int64_t p = 0; p < M; ++p) {
      double acc = +0.0;
      for (int64_t m = 0; m < K; ++m)
        acc = acc + G[p + m * ldg] * Y[m + c * ldy];
      Z[p + c * ldz] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Householder QR, Q^T application, triangular solve (Alg. 1 steps 2-3;     */
/* the paper uses GeQRF + OrMQR + a triangular solve, Sec. 6.1 and 6.3).     */
/* ------------------------------------------------------------------------ */

/*
 * In-place Householder QR of the m x n matrix W (m >= n), LAPACK geqr2
 * convention: for column j with alpha = W[j,j] and tail x = W[j+1:m, j],
 *   if ||x|| == 0: tau_j = 0 (the reflector is the identity);
 *   else beta = -sign(alpha)*sqrt(alpha^2 + ||x||^2), tau_j = (beta-alpha)/beta,
 *        v = [1; x/(alpha-beta)], W[j,j] = beta, W[j+1:m,j] = v[1:];
 *   then H_j = I - tau_j v v^T is applied to columns j+1..n-1.
 * On exit R is the upper triangle of W, the reflector tails sit below it.
 */
void or_householder_qr(int64_t m, int64_t n, double *W, int64_t ldw,
                       double *tau) {
  for (int64_t j = 0; j < n; ++j) {
    double *col = W + j * ldw;
    const double alpha = col[j];
    double xnorm2 = 0.0;
    for (int64_t i = j + 1; i < m; ++i) xnorm2 = xnorm2 + col[i] * col[i];
    if (xnorm2 == 0.0) {
      tau[j] = 0.0;
      continue;
    }
    const double norm = sqrt(alpha * alpha + xnorm2);
    const double beta = alpha >= 0.0 ? -norm : norm;
    tau[j] = (beta - alpha) / beta;
    const double scal = 1.0 / (alpha - beta);
    for (int64_t i = j + 1; i < m; ++i) col[i] = col[i] * scal;
    col[j] = beta;
    /* apply H_j to the trailing columns: C <- C - tau v (v^T C) */
    for (int64_t c = j + 1; c < n; ++c) {
      double *cc = W + c * ldw;
      double w = cc[j];
      for (int64_t i = j + 1; i < m; ++i) w = w + col[i] * cc[i];
      w = w * tau[j];
      cc[j] = cc[j] - w;
      for (int64_t i = j + 1; i < m; ++i) cc[i] = cc[i] - w * col[i];
    }
  }
}

/* B <- Q^T B = H_{n-1} ... H_1 H_0 B, with the reflectors left in W by
 * or_householder_qr (what OrMQR computes). */
void or_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *W,
                 int64_t ldw, const double *tau, double *B, int64_t ldb) {
  for (int64_t j = 0; j < n; ++j) {
    if (tau[j] == 0.0) continue;
    const double *v = W + j * ldw;
    for (int64_t c = 0; c < nrhs; ++c) {
      double *bc = B + c * ldb;
      double w = bc[j];
      for (int64_t i = j + 1; i < m; ++i) w = w + v[i] * bc[i];
      w = w * tau[j];
      bc[j] = bc[j] - w;
      for (int64_t i = j + 1; i < m; ++i) bc[i] = bc[i] - w * v[i];
    }
  }
}

/* Back substitution R X = B for the n x n upper triangle of R; B (n x nrhs)
 * is overwritten by X.  Returns ORACLE_ERR_SINGULAR, with X set to NaN, when
 * a diagonal entry is zero or not finite. */
int or_trsv_upper(int64_t n, int64_t nrhs, const double *R, int64_t ldr,
                  double *B, int64_t ldb) {
  for (int64_t i = 0; i < n; ++i) {
    const double r = R[i + i * ldr];
    if (r == 0.0 || !isfinite(r)) {
      for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t j = 0; j < n; ++j) B[j + c * ldb] = NAN;
      return ORACLE_ERR_SINGULAR;
    }
  }
  for (int64_t c = 0; c < nrhs; ++c) {
    double *x = B + c * ldb;
    for (int64_t i = n - 1; i >= 0; --i) {
      double acc = x[i];
      for (int64_t j = i + 1; j < n; ++j) acc = acc - R[i + j * ldr] * x[j];
      x[i] = acc / R[i + i * ldr];
    }
  }
  return ORACLE_OK;
}

/*
 * Least squares through Householder QR of an m x n matrix W with right-hand
 * sides Bm (m x nrhs): [Q,R] = qr(W,0), X = R^{-1} (Q^T B)_{0:n}.  W and Bm
 * are copied, the inputs are untouched.  This is Alg. 1 steps 2-3 applied to
 * a sketched system, and the plain QR least-squares solver when W = A.
 */
int or_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W,
                int64_t ldw, const double *Bm, int64_t ldb, double *X,
                int64_t ldx) {
  if (m < n) return ORACLE_ERR_ARG;
  double *Wc = (double *)malloc((size_t)(m * n + 1) * sizeof(double));
  double *Bc = (double *)malloc((size_t)(m * nrhs + 1) * sizeof(double));
  double *tau = (double *)malloc((size_t)(n + 1) * sizeof(double));
  if (!Wc || !Bc || !tau) {
    free(Wc);
    free(Bc);
    free(tau);
    return ORACLE_ERR_NOMEM;
  }
  for (int64_t c = 0; c < n; ++c)
    memcpy(Wc + c * m, W + c * ldw, (size_t)m * sizeof(double));
  for (int64_t c = 0; c < nrhs; ++c)
    memcpy(Bc + c * m, Bm + c * ldb, (size_t)m * sizeof(double));
  or_householder_qr(m, n, Wc, m, tau);
  or_apply_qt(m, n, nrhs, Wc, m, tau, Bc, m);
  int st = or_trsv_upper(n, nrhs, Wc, m, Bc, m);
  for (int64_t c = 0; c < nrhs; ++c)
    memcpy(X + c * ldx, Bc + c * m, (size_t)n * sizeof(double));
  free(Wc);
  free(Bc);
  free(tau);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Normal equations (Sec. 6.3: Gram by GEMM, A^T b by GEMV, Cholesky, two   */
/* triangular solves).  Comparator only.                                     */
/* ------------------------------------------------------------------------ */

int or_normal_equations(int64_t d, int64_t n, int64_t nrhs, const double *A,
                        int64_t lda, const double *B, int64_t ldb, double *X,
                        int64_t ldx) {
  double *Gm = (double *)malloc((size_t)(n * n + 1) * sizeof(double));
  if (!Gm) return ORACLE_ERR_NOMEM;
  for (int64_t q = 0; q < n; ++q)
    for (int64_t p = 0; p < n; ++p) {
      double acc = 0.0;
      for (int64_t i = 0; i < d; ++i)
        acc = acc + A[i + p * lda] * A[i + q * lda];
      Gm[p + q * n] = acc;
    }
  for (int64_t c = 0; c < nrhs; ++c)
    for (int64_t p = 0; p < n; ++p) {
      double acc = 0.0;
      for (int64_t i = 0; i < d; ++i)
        acc = acc + A[i + p * lda] * B[i + c * ldb];
      X[p + c * ldx] = acc;
    }
  /* Cholesky Gm = R^T R with R upper triangular, stored in the upper part */
  for (int64_t j = 0; j < n; ++j) {
    double diag = Gm[j + j * n];
    for (int64_t t = 0; t < j; ++t) diag = diag - Gm[t + j * n] * Gm[t + j * n];
    if (!(diag > 0.0) || !isfinite(diag)) {
      for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t p = 0; p < n; ++p) X[p + c * ldx] = NAN;
      free(Gm);
      return ORACLE_ERR_SINGULAR;
    }
    const double rjj = sqrt(diag);
    Gm[j + j * n] = rjj;
    for (int64_t q = j + 1; q < n; ++q) {
      double acc = Gm[j + q * n];
      for (int64_t t = 0; t < j; ++t) acc = acc - Gm[t + j * n] * Gm[t + q * n];
      Gm[j + q * n] = acc / rjj;
    }
  }
  for (int64_t c = 0; c < nrhs; ++c) {
    double *x = X + c * ldx;
    /* R^T y = A^T b (forward), then R x = y (backward) */
    for (int64_t i = 0; i < n; ++i) {
      double acc = x[i];
      for (int64_t t = 0; t < i; ++t) acc = acc - Gm[t + i * n] * x[t];
      x[i] = acc / Gm[i + i * n];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double acc = x[i];
      for (int64_t t = i + 1; t < n; ++t) acc = acc - Gm[i + t * n] * x[t];
      x[i] = acc / Gm[i + i * n];
    }
  }
  free(Gm);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Composite multisketch sketch-and-solve (Alg. 1 with S = G*C; Sec. 1      */
/* multisketch S2(S1 x), with S1 the CountSketch and S2 the Gaussian).       */
/* ------------------------------------------------------------------------ */

/*
 * X = argmin || G C (B - A X) || for FP64 A (d x n) and B (d x nrhs):
 *   Y = C [A | B]   (canonical CountSketch, FP64)
 *   Z = G Y         (k2 x (n+nrhs), FP64)
 *   [Q,R] = qr(Z_A), X = R^{-1} (Q^T Z_B)_{0:n}.
 * The association is G (C A), never (G C) A.  Ys (k x (n+nrhs)) and
 * Zs (k2 x (n+nrhs)) receive the intermediates when non-NULL.
 */
int or_sketch_lstsq_f64(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                        int64_t k2, const double *A, int64_t lda,
                        const double *B, int64_t ldb, const int32_t *h,
                        const int8_t *s, const double *G, int64_t ldg,
                        double *X, int64_t ldx, double *Ys, double *Zs) {
  if (k2 < n) return ORACLE_ERR_ARG;
  const int64_t nc = n + nrhs;
  double *Y = (double *)malloc((size_t)(k * nc + 1) * sizeof(double));
  double *Z = (double *)malloc((size_t)(k2 * nc + 1) * sizeof(double));
  if (!Y || !Z) {
    free(Y);
    free(Z);
    return ORACLE_ERR_NOMEM;
  }
  int st = or_countsketch_f64(d, n, k, A, lda, h, s, Y, k);
  if (st == ORACLE_OK)
    st = or_countsketch_f64(d, nrhs, k, B, ldb, h, s, Y + n * k, k);
  if (st == ORACLE_OK) {
    or_gemm_f64(k2, nc, k, G, ldg, Y, k, Z, k2);
    st = or_qr_solve(k2, n, nrhs, Z, k2, Z + n * k2, k2, X, ldx);
  }
  if (Ys && st != ORACLE_ERR_RANGE) memcpy(Ys, Y, (size_t)(k * nc) * sizeof(double));
  if (Zs && st != ORACLE_ERR_RANGE) memcpy(Zs, Z, (size_t)(k2 * nc) * sizeof(double));
  free(Y);
  free(Z);
  return st;
}

/* ------------------------------------------------------------------------ */
/* BF16 rounding (round to nearest, ties to even) of an FP32 value, returned */
/* as the FP32 value it denotes.  A BF16 number is the upper 16 bits of an   */
/* IEEE binary32; rounding keeps those bits after adding half an ulp of the  */
/* kept part, with ties going to the even kept pattern.  NaN stays NaN.      */
/* ------------------------------------------------------------------------ */

float or_round_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, sizeof u);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0) {
    u |= 0x00400000u; /* quiet NaN, keep the sign and payload top bits */
    u &= 0xffff0000u;
  } else {
    const uint32_t lsb = (u >> 16) & 1u;
    u = u + 0x7fffu + lsb;
    u &= 0xffff0000u;
  }
  float r;
  memcpy(&r, &u, sizeof r);
  return r;
}

/* Element-wise or_round_bf16 over an array. */
void or_round_bf16_array(int64_t count, const float *x, float *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = or_round_bf16(x[i]);
}

/* ------------------------------------------------------------------------ */
/* FP16 rounding (IEEE binary16: 11-bit significand, exponents -14..15,     */
/* subnormals spaced 2^-24, largest finite 65504), round to nearest, ties to */
/* even, of an FP32 value, returned as the FP32 value it denotes.  The      */
/* spacing of binary16 numbers around |x| in [2^(E-1), 2^E) is 2^(E-11),    */
/* never below 2^-24; |x| is rounded to a multiple of that spacing (exact   */
/* in FP64) and a result of 2^16 or more overflows to infinity.             */
/* ------------------------------------------------------------------------ */

float or_round_f16(float x) {
  if (isnan(x) || isinf(x)) return x;
  const double a = fabs((double)x);
  if (a == 0.0) return x;
  int E;
  frexp(a, &E); /* a = m 2^E, m in [0.5, 1) */
  int q = E - 11;
  if (q < -24) q = -24;
  const double r = ldexp(nearbyint(ldexp(a, -q)), q); /* ties to even */
  const float v = r >= 65536.0 ? INFINITY : (float)r;
  return x < 0.0f ? -v : v;
}

/* The FP16 Gaussian stage's column exponent: e = floor(log2 max_i |y_i|) -
 * 14 held in [-112, 112], so that 2^-e y has its largest magnitude in
 * [2^14, 2^15); 0 for a zero column or one holding a NaN or an infinity. */
int or_f16_col_exp(int64_t k, const float *y) {
  double m = 0.0;
  for (int64_t i = 0; i < k; ++i) {
    if (!isfinite(y[i])) return 0;
    const double a = fabs((double)y[i]);
    if (a > m) m = a;
  }
  if (m == 0.0) return 0;
  int E;
  frexp(m, &E); /* floor(log2 m) = E - 1 */
  int e = E - 1 - 14;
  if (e < -112) e = -112;
  if (e > 112) e = 112;
  return e;
}

/* Y (k x nc, FP32) as the FP16 Gaussian stage reads it: column c scaled by
 * 2^-e_c (an FP32 product), rounded to FP16, scaled back by 2^e_c (exact in
 * FP64).  out: k x nc FP64. */
void or_round_f16_colscaled(int64_t k, int64_t nc, const float *Y, int64_t ldy,
                            double *out, int64_t ldo) {
  for (int64_t c = 0; c < nc; ++c) {
    const float *y = Y + c * ldy;
    const int e = or_f16_col_exp(k, y);
    const float down = ldexpf(1.0f, -e);
    for (int64_t i = 0; i < k; ++i)
      out[i + c * ldo] = ldexp((double)or_round_f16(y[i] * down), e);
  }
}

/*
 * FP32 data path of the same composite: Y = C [A | B] folded in FP32; when
 * y_bf16 has ORACLE_Y_BF16 Y is rounded to BF16 (RNE) before the Gaussian
 * stage, with ORACLE_Y_F16 to FP16 after the column scaling of the FP16
 * stage (or_round_f16_colscaled);
 * Z = G Y is then formed in FP64 from the exact FP64 images of the FP32 (or
 * BF16) values and of G (G is passed as the FP64 images of its stored
 * values); QR and solve are FP64.
 */
int or_sketch_lstsq_f32(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                        int64_t k2, const float *A, int64_t lda,
                        const float *B, int64_t ldb, const int32_t *h,
                        const int8_t *s, const double *G, int64_t ldg,
                        int y_bf16, double *X, int64_t ldx, float *Ys,
                        double *Zs) {
  if (k2 < n) return ORACLE_ERR_ARG;
  const int64_t nc = n + nrhs;
  float *Y = (float *)malloc((size_t)(k * nc + 1) * sizeof(float));
  double *Yd = (double *)malloc((size_t)(k * nc + 1) * sizeof(double));
  double *Z = (double *)malloc((size_t)(k2 * nc + 1) * sizeof(double));
  if (!Y || !Yd || !Z) {
    free(Y);
    free(Yd);
    free(Z);
    return ORACLE_ERR_NOMEM;
  }
  int st;
  if (y_bf16 & ORACLE_Y_ACC64) {
    /* Def. 3's sums taken in FP64 (exact for these FP32 terms up to FP64
     * rounding) and rounded once to FP32: the FP32 sketch closest to the
     * exact one */
    st = or_countsketch_f32_acc64(d, n, k, A, lda, h, s, Yd, k);
    if (st == ORACLE_OK)
      st = or_countsketch_f32_acc64(d, nrhs, k, B, ldb, h, s, Yd + n * k, k);
    if (st == ORACLE_OK)
      for (int64_t t = 0; t < k * nc; ++t) Y[t] = (float)Yd[t];
  } else {
    st = or_countsketch_f32(d, n, k, A, lda, h, s, Y, k);
    if (st == ORACLE_OK)
      st = or_countsketch_f32(d, nrhs, k, B, ldb, h, s, Y + n * k, k);
  }
  if (st == ORACLE_OK) {
    if (y_bf16 & ORACLE_Y_F16)
      or_round_f16_colscaled(k, nc, Y, k, Yd, k);
    else
      for (int64_t t = 0; t < k * nc; ++t)
        Yd[t] = (double)((y_bf16 & ORACLE_Y_BF16) ? or_round_bf16(Y[t]) : Y[t]);
    or_gemm_f64(k2, nc, k, G, ldg, Yd, k, Z, k2);
    st = or_qr_solve(k2, n, nrhs, Z, k2, Z + n * k2, k2, X, ldx);
  }
  if (Ys && st != ORACLE_ERR_RANGE) memcpy(Ys, Y, (size_t)(k * nc) * sizeof(float));
  if (Zs && st != ORACLE_ERR_RANGE) memcpy(Zs, Z, (size_t)(k2 * nc) * sizeof(double));
  free(Y);
  free(Yd);
  free(Z);
  return st;
}

/* ------------------------------------------------------------------------ */
/* rand_cholQR least squares (Alg. 5, Sec. 6.3) with the multisketch S = G C */
/* as the sketch operator.  The steps in the paper's order:                 */
/*   1. Y = S A                 (CountSketch of A, then the Gaussian stage)  */
/*   2. R0 = R factor of the economy QR of Y (Householder)                   */
/*   3. Q0 = A R0^{-1}          (each row q of Q0 solves q R0 = a)           */
/*   4. Gm = Q0^T Q0, z = Q0^T B                                             */
/*   5. R1 = chol(Gm)           (upper, Gm = R1^T R1)                        */
/*   6. R = R1 R0                                                            */
/*   7. y = R1^{-T} z                                                        */
/*   8. x = R^{-1} y                                                         */
/* Q0 is never stored: each row is solved and folded into Gm and z in       */
/* ascending row order.  Y_f64 holds S A in FP64 (the caller's sketch of A  */
/* in whatever precision it was formed, promoted); A and B are FP64 (FP32   */
/* data promoted exactly by the caller).  R (n x n, upper, zeros below) is   */
/* written when Rout is not NULL.                                            */
/* ------------------------------------------------------------------------ */
int or_rand_cholqr_from_sketch(int64_t d, int64_t n, int64_t nrhs, int64_t m,
                               const double *SA, int64_t lds, const double *A,
                               int64_t lda, const double *B, int64_t ldb, double *X,
                               int64_t ldx, double *Rout, int64_t ldr) {
  if (m < n || n < 1) return ORACLE_ERR_ARG;
  double *W = (double *)malloc((size_t)(m * n) * sizeof(double));
  double *tau = (double *)malloc((size_t)n * sizeof(double));
  double *Gm = (double *)calloc((size_t)(n * n), sizeof(double));
  double *z = (double *)calloc((size_t)(n * (nrhs > 0 ? nrhs : 1)), sizeof(double));
  double *q = (double *)malloc((size_t)n * sizeof(double));
  double *R = (double *)calloc((size_t)(n * n), sizeof(double));
  int st = ORACLE_OK;
  if (!W || !tau || !Gm || !z || !q || !R) {
    st = ORACLE_ERR_NOMEM;
    goto done;
  }
  /* step 2: R0 in the upper triangle of W */
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i < m; ++i) W[i + c * m] = SA[i + c * lds];
  or_householder_qr(m, n, W, m, tau);
  for (int64_t j = 0; j < n; ++j)
    if (W[j + j * m] == 0.0 || !isfinite(W[j + j * m])) {
      st = ORACLE_ERR_SINGULAR;
      goto done;
    }
  /* steps 3-4: row i of Q0 by forward substitution, folded into Gm and z */
  for (int64_t i = 0; i < d; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      double acc = A[i + j * lda];
      for (int64_t l = 0; l < j; ++l) acc = acc - q[l] * W[l + j * m];
      q[j] = acc / W[j + j * m];
    }
    for (int64_t c2 = 0; c2 < n; ++c2)
      for (int64_t p = 0; p < n; ++p) Gm[p + c2 * n] = Gm[p + c2 * n] + q[p] * q[c2];
    for (int64_t c = 0; c < nrhs; ++c)
      for (int64_t p = 0; p < n; ++p) z[p + c * n] = z[p + c * n] + q[p] * B[i + c * ldb];
  }
  /* step 5: Cholesky Gm = R1^T R1, R1 in the upper triangle of Gm */
  for (int64_t j = 0; j < n; ++j) {
    double diag = Gm[j + j * n];
    for (int64_t t = 0; t < j; ++t) diag = diag - Gm[t + j * n] * Gm[t + j * n];
    if (!(diag > 0.0) || !isfinite(diag)) {
      st = ORACLE_ERR_SINGULAR;
      goto done;
    }
    const double rjj = sqrt(diag);
    Gm[j + j * n] = rjj;
    for (int64_t c2 = j + 1; c2 < n; ++c2) {
      double acc = Gm[j + c2 * n];
      for (int64_t t = 0; t < j; ++t) acc = acc - Gm[t + j * n] * Gm[t + c2 * n];
      Gm[j + c2 * n] = acc / rjj;
    }
  }
  /* step 6: R = R1 R0 (both upper triangular) */
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i <= j; ++i) {
      double acc = 0.0;
      for (int64_t t = i; t <= j; ++t) acc = acc + Gm[i + t * n] * W[t + j * m];
      R[i + j * n] = acc;
    }
  /* steps 7-8: R1^T y = z (forward), then R x = y (backward) */
  for (int64_t c = 0; c < nrhs; ++c) {
    double *y = z + c * n;
    for (int64_t i = 0; i < n; ++i) {
      double acc = y[i];
      for (int64_t t = 0; t < i; ++t) acc = acc - Gm[t + i * n] * y[t];
      y[i] = acc / Gm[i + i * n];
    }
    double *x = X + c * ldx;
    for (int64_t i = n - 1; i >= 0; --i) {
      double acc = y[i];
      for (int64_t t = i + 1; t < n; ++t) acc = acc - R[i + t * n] * x[t];
      x[i] = acc / R[i + i * n];
    }
  }
  if (Rout)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) Rout[i + j * ldr] = i <= j ? R[i + j * n] : 0.0;
done:
  if (st != ORACLE_OK && st != ORACLE_ERR_NOMEM)
    for (int64_t c = 0; c < nrhs; ++c)
      for (int64_t p = 0; p < n; ++p) X[p + c * ldx] = NAN;
  free(W);
  free(tau);
  free(Gm);
  free(z);
  free(q);
  free(R);
  return st;
}

/* ------------------------------------------------------------------------
 * Hash-generated CountSketch (Sec. 8 names it future work: the bucket and
 * sign of each row come from a hash of the row index instead of stored
 * vectors).  The hash is SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): the state advances by the
 * odd constant gamma = 0x9E3779B97F4A7C15 and each output is the state passed
 * through the finaliser mix64.  Row i (0-based) takes the (i+1)-th output of
 * the generator started at state `seed`:
 *   u_i = mix64(seed + (i + 1) gamma)   (mod 2^64)
 *   h_i = floor((u_i >> 32) k / 2^32)  (multiply-shift: 0 <= h_i < k)
 *   s_i = +1 if bit 0 of u_i is 0, else -1.
 * ------------------------------------------------------------------------ */
static uint64_t or_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);
  z = (z ^ (z >> 27)) * UINT64_C(0x94D049BB133111EB);
  return z ^ (z >> 31);
}

/* `count` successive SplitMix64 outputs from state `seed`. */
void or_splitmix64(uint64_t seed, int64_t count, uint64_t *out) {
  uint64_t state = seed;
  for (int64_t t = 0; t < count; ++t) {
    state = state + UINT64_C(0x9E3779B97F4A7C15);
    out[t] = or_mix64(state);
  }
}

/* h and s of rows 0 .. d-1 for k buckets (1 <= k <= 2^31). */
int or_hash_sketch(int64_t d, int64_t k, uint64_t seed, int32_t *h, int8_t *s) {
  if (d < 0 || k < 1 || k > (INT64_C(1) << 31)) return ORACLE_ERR_ARG;
  for (int64_t i = 0; i < d; ++i) {
    const uint64_t u = or_mix64(seed + (uint64_t)(i + 1) * UINT64_C(0x9E3779B97F4A7C15));
    h[i] = (int32_t)(((u >> 32) * (uint64_t)k) >> 32);
    s[i] = (u & 1) ? (int8_t)-1 : (int8_t)1;
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * SRHT (Sec. 5, its definition): S = k^{-1/2} P H_m D with H_m the Hadamard
 * matrix of the recursive definition, whose entries are
 *   H_m[a][b] = (-1)^{popcount(a AND b)}
 * (the block rule [[H, H], [H, -H]] adds one bit to both indices, and the
 * sign flips exactly when both new bits are 1), D = diag(dsign) and P
 * taking rows r_0 .. r_{k-1} of H_m D X.  m is the smallest power of two
 * >= the row count mx of X, which is padded with zero rows (the definition
 * needs log2 m integral).  Each output is that sum written out, accumulated
 * in long double, then scaled and rounded once:
 *   Y[j][c] = k^{-1/2} sum_{i < mx} (-1)^{popcount(r_j AND i)} dsign_i X[i][c].
 * ------------------------------------------------------------------------ */
static int or_parity64(uint64_t v) {
  int p = 0;
  while (v) {
    p ^= 1;
    v &= v - 1;
  }
  return p;
}

int or_srht(int64_t mx, int64_t ncols, int64_t k, const double *X, int64_t ldx,
            const int8_t *dsign, const int32_t *r, double *Y, int64_t ldy) {
  if (mx < 1 || ncols < 0 || k < 1 || ldx < mx || ldy < k) return ORACLE_ERR_ARG;
  int64_t m = 1;
  while (m < mx) m *= 2;
  for (int64_t i = 0; i < mx; ++i)
    if (dsign[i] != 1 && dsign[i] != -1) return ORACLE_ERR_RANGE;
  for (int64_t j = 0; j < k; ++j)
    if (r[j] < 0 || r[j] >= m) return ORACLE_ERR_RANGE;
  const long double scale = 1.0L / sqrtl((long double)k);
  for (int64_t c = 0; c < ncols; ++c)
    for (int64_t j = 0; j < k; ++j) {
      long double acc = 0.0L;
      for (int64_t i = 0; i < mx; ++i) {
        const long double v = (long double)dsign[i] * (long double)X[i + c * ldx];
        acc = or_parity64((uint64_t)r[j] & (uint64_t)i) ? acc - v : acc + v;
      }
      Y[j + c * ldy] = (double)(acc * scale);
    }
  return ORACLE_OK;
}

