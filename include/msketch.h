/*
 * msketch.h -- C ABI of the MI355X (gfx950) CountSketch / multisketch /
 * sketch-and-solve least-squares library (libmsketch.so).
 *
 * Method: Higgins, Boman, Yamazaki, "A High Performance GPU CountSketch
 * Implementation and Its Application to Multisketching and Least Squares
 * Problems" (arXiv 2508.14209).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller.  The library
 *    allocates no memory on any call; scratch space comes from the caller's
 *    workspace `ws` of `ws_bytes` bytes, sized by ms_workspace_size() and
 *    aligned to 256 bytes.
 *  - Matrices are column-major with a leading dimension (LAPACK style):
 *    element (i, j) of M is M[i + j*ldm], ldm >= number of rows.
 *  - The CountSketch S (k x d) of Def. 3 is given by a bucket map h (int32,
 *    0-based, h[i] in [0,k); the paper numbers buckets 1..k) and a sign s
 *    (int8, +1 or -1; the paper's boolean of Alg. 2 with true meaning +1).
 *    Column i of S is s[i] * e_{h[i]}.  S is never scaled.
 *  - The Gaussian stage matrix G (k2 x k) has N(0, 1/k2) entries (Sec. 1,
 *    variance 1/k2) and is passed in; h, s and G are data, so every result is
 *    reproducible from the seed that drew them.
 *  - Outputs are overwritten (accumulation starts from +0.0).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *    and runs asynchronously.  Argument errors are returned before anything
 *    is enqueued.  Errors found on the device (a bucket index outside [0,k),
 *    a sign that is not +-1, a zero or non-finite diagonal of R, a sorted-mode
 *    bucket longer than MS_SORTED_MAX_SEGMENT rows when k >
 *    MS_SORTED_BLOCKED_MAX_K) are recorded in a status
 *    word at the start of `ws` and returned by ms_check_status().  After such
 *    an error the outputs' contents are unspecified, except that a singular
 *    R leaves X filled with NaN.
 *  - Calls that share a workspace must be ordered (same stream or explicit
 *    synchronisation): the workspace is overwritten by every call.
 *  - Nothing throws across the ABI.
 */
#ifndef MSKETCH_H
#define MSKETCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MS_OK = 0,
  MS_ERR_ARG = 1,         /* invalid argument, detected on the host */
  MS_ERR_RANGE = 2,       /* h outside [0,k) or s not in {+1,-1} (device) */
  MS_ERR_NOMEM = 3,       /* workspace smaller than ms_workspace_size() */
  MS_ERR_SINGULAR = 4,    /* R has a zero or non-finite diagonal (device) */
  MS_ERR_DEVICE = 5,      /* a HIP runtime call or kernel launch failed */
  MS_ERR_UNSUPPORTED = 6  /* valid but unsupported combination or size */
} ms_status;

/* MS_BF16 and MS_F16 are passed as their 16-bit patterns (G only). */
typedef enum { MS_F64 = 0, MS_F32 = 1, MS_BF16 = 2, MS_F16 = 3 } ms_dtype;

/* How the CountSketch sum of Eq. (2) is formed on the device. */
typedef enum {
  MS_CS_AUTO = 0,   /* MS_CS_LDS */
  MS_CS_ATOMIC = 1, /* Alg. 2 as written: one global atomic add per element.
                       Measured baseline only. */
  MS_CS_LDS = 2,    /* coalesced streaming of A, per-workgroup bucket partial
                       sums in LDS, one flush per workgroup.  Summation order
                       varies from run to run. */
  MS_CS_SORTED = 3  /* deterministic: rows grouped by bucket by a stable
                       counting sort, each bucket folded in ascending row order
                       from +0.0 -- bit-identical to the sequential reading of
                       Alg. 2 */
} ms_cs_mode;

/* Longest bucket (rows sharing one h value) MS_CS_SORTED and ms_bucket_plan
   accept when k > MS_SORTED_BLOCKED_MAX_K (then each bucket is sorted on its
   own in LDS).  Up to MS_SORTED_BLOCKED_MAX_K buckets the plan is a blocked
   stable counting sort and a bucket may hold every row. */
#define MS_SORTED_MAX_SEGMENT 16384
#define MS_SORTED_BLOCKED_MAX_K 16384

typedef struct {
  int32_t cs_mode;      /* ms_cs_mode */
  int32_t refine_steps; /* sketch_lstsq: FP64-residual refinement steps */
  int32_t cs_tile_cols; /* MS_CS_LDS tuning: at most this many columns binned
                           per workgroup (power of two, 0 = automatic) */
  int32_t cs_schedule;  /* MS_CS_LDS tuning: 0 = persistent die-aware
                           schedule (default), 1 = one workgroup per (row
                           chunk, column tile, bucket tile) */
  int32_t batch_rows_log2;   /* sketch_lstsq_batched tuning: rows per
                                CountSketch work item = 2^x (0 = automatic,
                                else 8..24) */
  int32_t batch_kchunk_log2; /* sketch_lstsq_batched tuning: K per Gaussian-
                                stage work item = 2^x (0 = automatic, else
                                5..20) */
  int32_t gauss_y_terms;     /* BF16 / FP16 Gaussian stage
                                (multisketch_apply, sketch_lstsq,
                                rand_cholqr_lstsq, sketch_lstsq_batched):
                                1 = Y rounded to G's 16-bit format (nearest
                                even); 3 = Y split into three such terms
                                hi + mid + lo that sum to Y exactly (FP16:
                                down to 2^-40 of the column's largest
                                magnitude), so G Y is formed from the exact
                                Y with FP32 accumulation (three matrix-core
                                products per step, G read once); 0 = 3.
                                Other values: MS_ERR_ARG. */
  int32_t refine_tol_log2;   /* sketch_lstsq_batched: 0 = every problem takes
                                all refine_steps; x in 1..60 = a problem
                                stops refining once a step's correction dx
                                has ||dx||_F <= 2^-x ||X||_F (X after the
                                step); the later steps skip it.  Other
                                values: MS_ERR_ARG.  sketch_lstsq runs all
                                steps. */
} ms_opts;

/* op codes of ms_workspace_size() */
#define MS_OP_BUCKET_PLAN 0
#define MS_OP_COUNTSKETCH 1
#define MS_OP_GAUSSIAN 2
#define MS_OP_MULTISKETCH 3
#define MS_OP_QR_SOLVE 4
#define MS_OP_LSTSQ 5
#define MS_OP_RAND_CHOLQR 6
#define MS_OP_NORMAL_EQUATIONS 7
#define MS_OP_COUNTSKETCH_HASHED 8
#define MS_OP_SRHT 9
#define MS_OP_COUNT_SRHT_LSTSQ 10

/*
 * Bytes of workspace the operation needs (a multiple of 256, at least 256).
 * Arguments not used by `op` are ignored.  opts may be NULL (defaults).
 * Returns 0 for invalid arguments.
 */
size_t ms_workspace_size(int op, int64_t d, int64_t n, int64_t nrhs, int64_t k,
                         int64_t k2, ms_dtype a_dtype, ms_dtype g_dtype,
                         const ms_opts *opts);

/*
 * Synchronises `stream` and returns the device-side status recorded by the
 * last call that used `ws` (MS_OK if none).  The only entry point that blocks.
 */
ms_status ms_check_status(const void *ws, void *stream);

/* Human-readable name of a status code (static string). */
const char *ms_status_string(ms_status st);

/*
 * Sketch plan (bucket histogram, exclusive scan, stable counting sort).
 * The paper notes that the parallel fold of Alg. 2 needs atomic row
 * additions (Sec. 4); the plan instead groups rows by bucket.
 *   cnt[m]  = #{i : h[i] = m}                      (k entries, int32)
 *   off[m]  = cnt[0] + ... + cnt[m-1], off[k] = d  (k+1 entries, int32)
 *   perm    = the rows of bucket 0, then of bucket 1, ..., each group in
 *             ascending row order                  (d entries, int32)
 * Requires 0 <= d < 2^31, 1 <= k < 2^31.  h out of range -> MS_ERR_RANGE on
 * the device.  For k > MS_SORTED_BLOCKED_MAX_K a bucket longer than
 * MS_SORTED_MAX_SEGMENT rows records MS_ERR_UNSUPPORTED (its rows are then
 * left unsorted).  ws: ms_workspace_size(MS_OP_BUCKET_PLAN, d, 0, 0, k, ...).
 */
ms_status ms_bucket_plan(int64_t d, int64_t k, const int32_t *h, int32_t *cnt,
                         int32_t *off, int32_t *perm, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Packed sketch: validates (h, s) and stores one 32-bit word per row,
 *   code[i] = h[i] | (s[i] == -1 ? 0x80000000 : 0),
 * reusable by every countsketch_accumulate() call with the same sketch (the
 * CountSketch of Def. 3 is fixed once r and sigma are drawn).  Requires
 * 1 <= k < 2^31.  A row with h outside [0,k) or s not +-1 records
 * MS_ERR_RANGE on the device and is packed as bucket 0 with sign +1.
 * ws: any workspace of at least 256 bytes (only the status word is used).
 */
ms_status ms_pack_sketch(int64_t d, int64_t k, const int32_t *h, const int8_t *s,
                         uint32_t *code, void *ws, size_t ws_bytes, void *stream);

/*
 * Streaming accumulation Y += S A with a packed sketch (code from
 * ms_pack_sketch).  Y is NOT cleared, so a sketch of a tall matrix can be
 * built block of rows by block of rows, as the row-block sum
 * C A = sum_i C^(i) A^(i) of Sec. 7 (pass the codes of each block's rows).
 *   A: d x n (F64 or F32), lda >= max(1,d); Y: k x n (same dtype), ldy >= k.
 * opts->cs_mode: MS_CS_AUTO/MS_CS_LDS or MS_CS_ATOMIC; MS_CS_SORTED returns
 * MS_ERR_UNSUPPORTED (its fixed fold order starts from +0.0).  A code whose
 * bucket is >= k is skipped and recorded as MS_ERR_RANGE.
 * ws: at least 256 bytes (the status word).  A workspace of
 * ms_workspace_size(MS_OP_COUNTSKETCH, d, n, 0, k, 0, a_dtype, ...) bytes
 * also holds, after the status block, the per-die partial sums that the LDS
 * variant uses instead of atomic flushes when k is large next to d (then
 * 8 k n elements); with a smaller workspace that variant flushes with
 * atomics.
 */
ms_status countsketch_accumulate(int64_t d, int64_t n, int64_t k, ms_dtype a_dtype,
                                 const void *A, int64_t lda, const uint32_t *code, void *Y,
                                 int64_t ldy, const ms_opts *opts, void *ws,
                                 size_t ws_bytes, void *stream);

/*
 * CountSketch Y = S A (Def. 3, Eq. (2), Alg. 2).
 *   A: d x n, a_dtype MS_F64 or MS_F32, lda >= max(1,d).
 *   Y: k x n, same dtype as A, ldy >= k.  The atomic and sorted variants
 *   accumulate in A's precision; the LDS variant sums each workgroup's rows
 *   in FP64 and adds that partial sum to Y in Y's precision.
 *   h, s: d entries each (see the conventions above).
 * opts->cs_mode selects the variant; MS_CS_SORTED reproduces the ascending
 * row fold bit for bit.  d may be 0 (Y = 0).  n may be 0 (no-op).
 */
ms_status countsketch_apply(int64_t d, int64_t n, int64_t k, ms_dtype a_dtype,
                            const void *A, int64_t lda, const int32_t *h,
                            const int8_t *s, void *Y, int64_t ldy,
                            const ms_opts *opts, void *ws, size_t ws_bytes,
                            void *stream);

/*
 * Gaussian stage alone: Z = G Y (the second sketch of the multisketch
 * S2(S1 x), Sec. 1; k2 x k times k x ncols).
 *   (g_dtype, y_dtype) = (F64, F64): FP64 MFMA, Z is FP64.
 *                        (F32, F32): FP32 MFMA, Z is FP32.
 *                        (BF16, F32): Y rounded to BF16 (round to nearest
 *                        even), BF16 MFMA with FP32 accumulation, Z is FP32.
 *                        (F16, F32): column c of Y scaled by 2^-e_c,
 *                        e_c = floor(log2 max_i |Y[i,c]|) - 14 held in
 *                        [-112, 112] (0 for a zero or non-finite column),
 *                        rounded to FP16 (nearest even), FP16 MFMA with
 *                        FP32 accumulation, column c of the product
 *                        multiplied by 2^e_c; Z is FP32.
 *   G: k2 x k (BF16 and FP16 are passed as their 16-bit patterns),
 *   ldg >= k2.
 *   Y: k x ncols, ldy >= k.   Z: k2 x ncols, ldz >= k2.
 */
ms_status ms_gaussian_apply(int64_t k, int64_t ncols, int64_t k2,
                            ms_dtype g_dtype, const void *G, int64_t ldg,
                            ms_dtype y_dtype, const void *Y, int64_t ldy,
                            void *Z, int64_t ldz, void *ws, size_t ws_bytes,
                            void *stream);

/*
 * Multisketch Z = G (S A) (Sec. 1; Table 1 "MultiSketch"), always in that
 * association: the CountSketch first, then the Gaussian stage.
 *   a_dtype F64 -> g_dtype F64, Z FP64;  a_dtype F32 -> g_dtype F32, BF16 or
 *   F16 (the 16-bit stages as in ms_gaussian_apply, with opts->gauss_y_terms),
 *   Z FP32.  Z: k2 x n, ldz >= k2.  Requires k2 >= 1.
 */
ms_status multisketch_apply(int64_t d, int64_t n, int64_t k, int64_t k2,
                            ms_dtype a_dtype, const void *A, int64_t lda,
                            const int32_t *h, const int8_t *s, ms_dtype g_dtype,
                            const void *G, int64_t ldg, void *Z, int64_t ldz,
                            const ms_opts *opts, void *ws, size_t ws_bytes,
                            void *stream);

/*
 * Householder QR least squares of a small system (Alg. 1 steps 2-3, done in
 * the paper with GeQRF + OrMQR + a triangular solve, Sec. 6.1 and 6.3):
 *   [Q,R] = qr(W,0) with W m x n (m >= n), X = R^{-1} (Q^T Bm)_{0:n}.
 * FP64 throughout, LAPACK geqr2 reflector convention.
 *   W: m x n, ldw >= m.  Bm: m x nrhs, ldb >= m.  X: n x nrhs, ldx >= n.
 *   R: optional (may be NULL) n x n output of the triangular factor, ldr >= n
 *   (its strictly lower part is set to 0).
 * A zero or non-finite R diagonal -> MS_ERR_SINGULAR (device) and X = NaN.
 */
ms_status ms_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W,
                      int64_t ldw, const double *Bm, int64_t ldb, double *X,
                      int64_t ldx, double *R, int64_t ldr, void *ws,
                      size_t ws_bytes, void *stream);

/*
 * Multisketch sketch-and-solve least squares (Alg. 1 with S = G C):
 *   X = argmin || G C (B - A X) ||,  A d x n, B d x nrhs, X n x nrhs (FP64).
 * Steps: Y = C [A | B] (CountSketch, A's precision); Z = G Y (Gaussian stage,
 * MFMA in the precision of g_dtype); Householder QR of Z_A (k2 x n, FP64);
 * Q^T applied to Z_B; back substitution.
 *   a_dtype F64: g_dtype F64.   a_dtype F32: g_dtype F32, BF16 or F16.
 *   Requires d >= 1, n >= 1, nrhs >= 1, k >= 1, k2 >= n.
 * opts->refine_steps > 0 (requires nrhs <= 8) then repeats, in FP64,
 *   r = B - A X;  X += R^{-1} Q^T G (C r)
 * with the Q and R of the first pass.
 */
ms_status sketch_lstsq(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                       int64_t k2, ms_dtype a_dtype, const void *A, int64_t lda,
                       const void *B, int64_t ldb, const int32_t *h,
                       const int8_t *s, ms_dtype g_dtype, const void *G,
                       int64_t ldg, double *X, int64_t ldx,
                       const ms_opts *opts, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * sketch_lstsq for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the same computation, arguments and limits as sketch_lstsq, with no
 * workspace argument.  Its scratch space is a static device array of
 * MS_NOALLOC_SCRATCH_BYTES bytes per GPU, created with the library's code
 * object on each device it runs on and held until the process ends; the call
 * allocates nothing.
 *   status: optional device pointer (may be NULL) that receives, in stream
 *   order after the solve, the device-side status that ms_check_status would
 *   report for sketch_lstsq (MS_ERR_RANGE, MS_ERR_SINGULAR, ...).
 * Returns MS_ERR_NOMEM, before anything is enqueued, when the problem needs
 * more scratch than that (ms_workspace_size(MS_OP_LSTSQ, ...) >
 * MS_NOALLOC_SCRATCH_BYTES; e.g. 4,194,304 x 64 FP64 with k = 8192 and no
 * refinement needs 24.3 MiB), and MS_ERR_DEVICE when the array's device
 * address cannot be obtained.  Every call on a GPU uses that GPU's one array:
 * calls that overlap on the same GPU (streams not ordered with each other)
 * race and give undefined results; order them.
 */
#define MS_NOALLOC_SCRATCH_BYTES (32 << 20)
ms_status sketch_lstsq_noalloc(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                               int64_t k2, ms_dtype a_dtype, const void *A,
                               int64_t lda, const void *B, int64_t ldb,
                               const int32_t *h, const int8_t *s,
                               ms_dtype g_dtype, const void *G, int64_t ldg,
                               double *X, int64_t ldx, int32_t *status,
                               const ms_opts *opts, void *stream);

/*
 * rand_cholQR least squares (Alg. 5, Sec. 6.3) with the multisketch S = G C
 * as the sketch operator: X = argmin ||B - A X||, the least-squares optimum
 * itself (the sketch only preconditions; no O(1) distortion as in
 * sketch_lstsq).  Steps: Y = S A (CountSketch of A in its precision, then
 * the Gaussian stage), R0 = the R factor of the Householder QR of Y,
 * Q0 = A R0^{-1}, Q0^T Q0 and Q0^T B in FP64 in one pass over A and B
 * (FP32 data promoted exactly; Q0 is not stored up to n = 64),
 * R1 = chol(Q0^T Q0),
 * R = R1 R0, y = R1^{-T} Q0^T B, X = R^{-1} y.  Stable for kappa(A) < 1/u
 * (Sec. 6.3); the FP32 / BF16 sketch of an FP32 A changes only the
 * preconditioner, so X is the FP64 optimum for the stored data.
 *   Arguments as for sketch_lstsq, plus R (may be NULL): n x n (ld ldr >= n),
 *   receives R (upper triangular, zeros below; A = Q R with Q = A R^{-1}).
 *   opts->refine_steps must be 0.
 * Limits: n <= 256, nrhs <= 16, n + nrhs <= 272 (else MS_ERR_UNSUPPORTED).
 * Beyond n = 64 or n + nrhs = 80, Q0 is formed on matrix cores and stored
 * (d x n FP64 in the workspace) and its Gram product is a second pass.
 * Device status:
 * MS_ERR_SINGULAR (X = NaN) when R0 or the Cholesky factor breaks down,
 * MS_ERR_RANGE for h or s out of range.
 * ws: ms_workspace_size(MS_OP_RAND_CHOLQR, d, n, nrhs, k, k2, a_dtype,
 * g_dtype, opts) bytes.
 */
ms_status rand_cholqr_lstsq(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                            int64_t k2, ms_dtype a_dtype, const void *A,
                            int64_t lda, const void *B, int64_t ldb,
                            const int32_t *h, const int8_t *s, ms_dtype g_dtype,
                            const void *G, int64_t ldg, double *X, int64_t ldx,
                            double *R, int64_t ldr, const ms_opts *opts, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * Hash-generated CountSketch (Sec. 8 names it future work): Y = C A with the
 * bucket and sign of each row computed from (seed, row) instead of read from
 * stored h and s, which removes their 5 bytes per row of traffic and the
 * packing pass.  Row i (0-based) takes u = the (i+1)-th output of SplitMix64
 * started at state `seed` (Steele, Lea and Flood, OOPSLA 2014: the state
 * advances by 0x9E3779B97F4A7C15, the output is the state through its
 * finaliser); h_i = floor((u >> 32) k / 2^32), s_i = -1 if bit 0 of u is 1,
 * else +1.  ms_hash_sketch writes the same h and s, so
 * countsketch_apply(..., h, s, ...) computes the same sketch.
 *   d x n A (a_dtype MS_F64 or MS_F32, column-major, lda >= d), Y k x n of
 *   A's dtype (ldy >= k), overwritten.  1 <= k <= 2^31 - 2.
 *   opts: cs_mode MS_CS_AUTO or MS_CS_LDS and cs_schedule 0 only (else
 *   MS_ERR_UNSUPPORTED); cs_tile_cols as for countsketch_apply.
 *   Accumulation order as MS_CS_LDS (FP64 partial sums; not bit-stable).
 * ws: ms_workspace_size(MS_OP_COUNTSKETCH_HASHED, d, n, 0, k, 0, a_dtype,
 * a_dtype, opts) bytes.
 */
ms_status countsketch_hashed(int64_t d, int64_t n, int64_t k, uint64_t seed,
                             ms_dtype a_dtype, const void *A, int64_t lda,
                             void *Y, int64_t ldy, const ms_opts *opts,
                             void *ws, size_t ws_bytes, void *stream);

/*
 * h (d int32) and s (d int8) of the hash-generated CountSketch with this
 * seed and k (see countsketch_hashed); device pointers, written on `stream`.
 */
ms_status ms_hash_sketch(int64_t d, int64_t k, uint64_t seed, int32_t *h,
                         int8_t *s, void *stream);

/*
 * SRHT (Sec. 5): Y = k^{-1/2} P H_m D X, with H_m the Hadamard matrix of the
 * recursive definition (entries (-1)^popcount(a AND b)), m the smallest power
 * of two >= the m rows of X (X padded with zero rows; the definition needs
 * log2 m integral), D = diag(dsign) and P taking rows r[0..k-1] of H_m D X.
 *   X: m x ncols (x_dtype MS_F64 or MS_F32, column-major, ldx >= m);
 *   dsign: m int8, each +1 or -1; r: k int32, each in [0, padded m) (rows may
 *   repeat: P samples with replacement); Y: k x ncols FP64 (ldy >= k),
 *   overwritten.  1 <= m <= 2^31 - 2, ncols <= 65535, 1 <= k <= 2^24.
 * Device status MS_ERR_RANGE for a sign not +-1 or a row index out of range
 * (the offending entries then contribute zero).  One pass over X; the sum
 * over 8192-row blocks is taken in block order (repeatable bits).
 * ws: ms_workspace_size(MS_OP_SRHT, m, ncols, 0, k, 0, x_dtype, 0, NULL).
 */
ms_status srht_apply(int64_t m, int64_t ncols, int64_t k, ms_dtype x_dtype,
                     const void *X, int64_t ldx, const int8_t *dsign,
                     const int32_t *r, double *Y, int64_t ldy, void *ws,
                     size_t ws_bytes, void *stream);

/*
 * Sketch-and-solve (Alg. 1) with the Count + SRHT multisketch (Sec. 8 names
 * it future work): Z = S2 (C [A | B]) with C the CountSketch (h, s; k1
 * buckets, accumulated in A's precision as in sketch_lstsq) and S2 the SRHT
 * of its k1 rows (dsign: k1 int8; r: k2 int32 in [0, padded k1)), in FP64;
 * then the Householder QR of Z's first n columns and X = R^{-1} (Q^T Z_B).
 *   Other arguments as for sketch_lstsq; k2 >= n; opts->refine_steps must
 *   be 0.  Device status as for sketch_lstsq and srht_apply.
 * ws: ms_workspace_size(MS_OP_COUNT_SRHT_LSTSQ, d, n, nrhs, k1, k2, a_dtype,
 * 0, opts) bytes.
 */
ms_status count_srht_lstsq(int64_t d, int64_t n, int64_t nrhs, int64_t k1,
                           int64_t k2, ms_dtype a_dtype, const void *A,
                           int64_t lda, const void *B, int64_t ldb,
                           const int32_t *h, const int8_t *s,
                           const int8_t *dsign, const int32_t *r, double *X,
                           int64_t ldx, const ms_opts *opts, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * Least squares by the normal equations (Sec. 6.3: the deterministic solver
 * the paper measures sketch-and-solve against): W = [A | B]^T [A | B] in
 * FP64 in one pass over A and B (FP32 data promoted exactly; a fixed
 * summation order, so results repeat bit for bit), R = chol(A^T A),
 * R^T y = A^T B, X = R^{-1} y.  Accurate only while kappa(A) is well below
 * u^{-1/2} (the Gram matrix squares the condition number; Sec. 6.3).
 *   d x n A (a_dtype MS_F64 or MS_F32, column-major, lda >= d), d x nrhs B
 *   (A's dtype, ldb >= d), X n x nrhs FP64 (ldx >= n); R (may be NULL):
 *   n x n (ldr >= n), receives R (upper triangular, zeros below).
 *   opts is unused (may be NULL).
 * Limits: n <= 256, nrhs <= 16, n + nrhs <= 272 (else MS_ERR_UNSUPPORTED).
 * Up to 64 columns (n + nrhs <= 80) one fused pass accumulates the Gram
 * matrix in registers; wider problems take a tiled Gram pass (per-chunk
 * partials of its upper 16 x 16 tiles, summed in chunk order) and a blocked
 * Cholesky (64 x 64 blocks).  Device status:
 * MS_ERR_SINGULAR (X = NaN) when the Cholesky factorisation breaks down.
 * ws: ms_workspace_size(MS_OP_NORMAL_EQUATIONS, d, n, nrhs, 0, 0, a_dtype,
 * 0, NULL) bytes.
 */
ms_status normal_equations_lstsq(int64_t d, int64_t n, int64_t nrhs,
                                 ms_dtype a_dtype, const void *A, int64_t lda,
                                 const void *B, int64_t ldb, double *X,
                                 int64_t ldx, double *R, int64_t ldr,
                                 const ms_opts *opts, void *ws, size_t ws_bytes,
                                 void *stream);

/*
 * One problem of a batched multisketch sketch-and-solve (all device
 * pointers; the meaning of every field is that of the sketch_lstsq argument
 * of the same name).
 */
typedef struct {
  int64_t d, n, nrhs, k, k2;
  const void *A;
  int64_t lda;
  const void *B;
  int64_t ldb;
  const int32_t *h;
  const int8_t *s;
  const void *G;
  int64_t ldg;
  double *X;
  int64_t ldx;
} ms_problem;

/* Largest sketched system a batched problem may have (register-resident QR). */
#define MS_BATCH_MAX_K2 256
#define MS_BATCH_MAX_COLS 144

/*
 * Workspace bytes of sketch_lstsq_batched for these problems (host array).
 * 0 for invalid arguments.  A workspace sized for one set of problems serves
 * any other set with the same count whose problems are no larger in k,
 * k2 and n + nrhs (and, with refinement, in d * nrhs).  Without refinement
 * d enters only through the packed bucket words (4 bytes per row, written
 * once per call): a set with more rows in total than the sizing set still
 * runs, reading h and s in every CountSketch work item instead (slower).
 */
size_t ms_batch_workspace_size(int count, const ms_problem *probs,
                               ms_dtype a_dtype, ms_dtype g_dtype,
                               const ms_opts *opts);

/*
 * Batched multisketch sketch-and-solve: every problem p is solved as
 * sketch_lstsq would solve it (same association G (C [A | B]), same
 * Householder QR and back substitution, same FP64-residual refinement), all
 * problems together in a fixed sequence of launches (seven, plus five per
 * refinement step) whose grids do not depend on the problems' contents -- so
 * the sequence can be captured once in a HIP graph and replayed after the
 * descriptors in device memory are rewritten.
 *   count      number of problems (1 .. 65535);
 *   probs_host host copy of the descriptors: validated, and used for the
 *              launch shapes (LDS size, QR register tile);
 *   probs_dev  the same descriptors in device memory (read by the kernels);
 *   a_dtype    MS_F32 or MS_F64 (all problems); g_dtype as for sketch_lstsq
 *              except MS_F16 (MS_ERR_UNSUPPORTED).
 * Limits per problem: k2 <= MS_BATCH_MAX_K2, n + nrhs <= MS_BATCH_MAX_COLS,
 * k2 >= n >= 1, nrhs >= 1, 1 <= d < 2^31, 1 <= k < 2^31.  The CountSketch is the
 * LDS variant (MS_CS_AUTO / MS_CS_LDS; MS_CS_ATOMIC -> MS_ERR_UNSUPPORTED) or,
 * with opts->cs_mode MS_CS_SORTED, the deterministic one: every bucket sum
 * folded in ascending row order in A's precision (the sequential reading of
 * Alg. 2, as sketch_lstsq's MS_CS_SORTED), so that -- with the other options
 * fixed -- each problem's X is bit-identical whatever else is in the batch
 * (every other stage of a problem depends on that problem alone); requires
 * k < 2^19 (else the problem is invalid: MS_ERR_ARG).
 * opts->refine_steps (0 .. 64) refinement steps
 * x <- x + R^{-1} Q^T G C (b - A x) with the FP64 residual, as in
 * sketch_lstsq; with refinement every problem needs nrhs <= 8 (else
 * MS_ERR_UNSUPPORTED).  Device errors are recorded per problem
 * (ms_batch_status) and in the workspace status word.
 */
ms_status sketch_lstsq_batched(int count, const ms_problem *probs_host,
                               const ms_problem *probs_dev, ms_dtype a_dtype,
                               ms_dtype g_dtype, const ms_opts *opts, void *ws,
                               size_t ws_bytes, void *stream);

/* Synchronises `stream` and copies the per-problem status codes of the last
 * sketch_lstsq_batched call on `ws` into status_host (count entries). */
ms_status ms_batch_status(const void *ws, int count, int32_t *status_host,
                          void *stream);

/*
 * Synthetic least-squares request generated on the device from a seed: a
 * matrix of prescribed condition number, as in the experiments of Sec. 6.3
 * (there kappa(A) = 1e2, or swept), for the serving workload, whose inputs
 * arrive faster than a host could upload them.  Not a step of the method.
 *   A (d x n FP32, column-major, lda >= d) = Z diag(D) Q: Z with independent
 *     N(0,1) entries, D_j = kappa^(-j/(n-1)) (D_0 = 1), Q = (I - 2 u1 u1^T)
 *     (I - 2 u2 u2^T) with unit Gaussian directions u1, u2;
 *   xstar (n x nrhs FP32, ld n) N(0,1);
 *   B (d x nrhs FP32, ldb >= d) = A xstar + noise * N(0,1) (needs A);
 *   h (d int32) uniform in [0, k), s (d int8) uniform in {-1, +1} (both or
 *     neither);
 *   G (k2 x k, column-major, ld k2; g_dtype MS_F32, MS_BF16 (rounded to
 *     nearest even) or MS_F64 (exact)) = N(0,1) / sqrt(k2) drawn in FP32.
 * Device pointers, written on `stream`; any output may be NULL (not made).
 * Limits: d >= 1, 1 <= n <= 128, 1 <= nrhs <= 8, 1 <= k, k2 <= 2^31 - 2,
 * kappa >= 1 and finite (else MS_ERR_ARG).  Each value depends only on the
 * seed and its position (counter-based SplitMix64 words, Box-Muller normals),
 * so a seed gives the same request on any device or stream.
 */
ms_status ms_gen_lstsq_request(uint64_t seed, int64_t d, int64_t n, int64_t nrhs,
                               double kappa, double noise, int64_t k, int64_t k2,
                               ms_dtype g_dtype, float *A, int64_t lda, float *B,
                               int64_t ldb, float *xstar, int32_t *h, int8_t *s,
                               void *G, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MSKETCH_H */
