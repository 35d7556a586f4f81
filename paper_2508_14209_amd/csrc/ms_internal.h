// ms_internal.h -- shared declarations of libmsketch's HIP translation units.
//
// Device helpers, the workspace layout and the host-side launchers each
// kernel file exports to the C-ABI layer (api.hip).  Nothing here is part of
// the public ABI (include/msketch.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "msketch.h"

namespace ms {

// ---------------------------------------------------------------- device info
struct DevInfo {
  int cus = 0;            // compute units
  int lds_per_block = 0;  // bytes of LDS one workgroup may allocate
  int xcds = 8;           // accelerator complex dies (L2 domains)
};
// Properties of the current device, queried once per device and cached.
const DevInfo &dev_info();
// Raise a kernel's dynamic-LDS limit once per (kernel, device).
hipError_t allow_dynamic_lds(const void *kernel, int bytes);

// ---------------------------------------------------------------- status word
// The first 256 bytes of every workspace hold an int32 status; kernels record
// the first device-side error with a compare-and-swap from MS_OK.
__device__ inline void record_status(int *st, int code) {
  atomicCAS(st, (int)MS_OK, code);
}

// ---------------------------------------------------------------- sign codes
// A row's bucket and sign packed in one word: bits 0..30 hold h[i], bit 31 is
// set when s[i] = -1.  The same packing carries a row index and its sign in
// the sorted plan.
constexpr uint32_t kSignBit = 0x80000000u;
constexpr uint32_t kIdxMask = 0x7fffffffu;

// +-a selected by the sign bit of `code`: flipping the IEEE sign bit is exact
// negation, so this is the add-or-subtract of Alg. 2 with no multiply.
__device__ __forceinline__ float apply_sign(float a, uint32_t code) {
  return __uint_as_float(__float_as_uint(a) ^ (code & kSignBit));
}
__device__ __forceinline__ double apply_sign(double a, uint32_t code) {
  uint64_t u = (uint64_t)__double_as_longlong(a) ^ ((uint64_t)(code & kSignBit) << 32);
  return __longlong_as_double((long long)u);
}

// ---------------------------------------------------------------- workspace
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline size_t dtype_size(ms_dtype t) {
  return t == MS_F64 ? 8 : t == MS_F32 ? 4 : 2;
}

// Bump allocator over the caller's workspace (offsets only; no allocation).
struct Carve {
  size_t off = kAlign;  // the status word occupies the first block
  size_t take(size_t bytes) {
    size_t o = off;
    off += align_up(bytes ? bytes : 1);
    return o;
  }
};

// Loads through a global-address-space pointer.  A pointer read from memory
// (a batch descriptor) is generic to the compiler, and loads through it are
// flat loads, which also count against the LDS wait counter: every wait for
// an LDS operation then waits for the outstanding memory loads too.  Every
// device pointer handed to this library addresses global memory, so the
// cast at the load is exact; the compiler then issues global loads.
template <typename T>
__device__ __forceinline__ T gload(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ T gload_nt(const T *p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)p);
}

// ---------------------------------------------------------------- launchers
// Columns of the sketched operand [A | B]: column c < n_a is A's column c,
// the rest are B's.  B may be null when n_a == ncols.
template <typename T>
struct Cols {
  const T *A;
  int64_t lda;
  const T *B;
  int64_t ldb;
  int n_a;
  int ncols;
  // the hash-generated sketch: rows' buckets and signs come from (key, row)
  // instead of stored vectors (LDS CountSketch only)
  int hashed = 0;
  uint64_t key = 0;
};

// countsketch.hip
hipError_t launch_zero_status(int *status, hipStream_t st);
// Clear the status word and a rows x cols buffer (ld) in one launch.
template <typename T>
hipError_t launch_prologue(int *status, T *Y, int64_t rows, int64_t cols, int64_t ld,
                           hipStream_t st);
template <typename T>
hipError_t launch_fill_zero(T *Y, int64_t rows, int64_t cols, int64_t ld, hipStream_t st);
hipError_t launch_pack_codes(int64_t d, int64_t k, const int32_t *h, const int8_t *s,
                             uint32_t *code, int *status, hipStream_t st);
// Plan: cnt (k, zero on entry), off (k+1), cursor (k), sperm (d) -- row
// index | sign bit (sign bit only when s is non-null).
hipError_t launch_plan(int64_t d, int64_t k, const int32_t *h, const int8_t *s,
                       int32_t *cnt, int32_t *off, int32_t *cursor, uint32_t *sperm,
                       int *status, hipStream_t st);
hipError_t launch_strip_sign(int64_t d, const uint32_t *sperm, int32_t *perm, hipStream_t st);

// zero_first: clear Y before accumulating (false: Y += S [A | B]).  status
// receives MS_ERR_RANGE for a code whose bucket is >= k (such rows are skipped).
template <typename T>
hipError_t launch_cs_atomic(int64_t d, int64_t k, const Cols<T> &c, const uint32_t *code,
                            T *Y, int64_t ldy, bool zero_first, int *status, hipStream_t st);
// Tuning of the LDS CountSketch (zero fields: defaults).
struct CsTuning {
  int cols_per_wg;   // upper bound on the columns one workgroup bins at once
  int grid_variant;  // 1: one workgroup per (row chunk, column tile, bucket tile)
};
// LDS variant: the bucket/sign words come from `code` when non-null, else
// from h and s directly (validated in the kernel).
template <typename T>
hipError_t launch_cs_lds(int64_t d, int64_t k, const Cols<T> &c, const uint32_t *code,
                         const int32_t *h, const int8_t *s, T *Y, int64_t ldy, bool zero_first,
                         int *status, hipStream_t st, const CsTuning *tune = nullptr,
                         void *part = nullptr, size_t part_bytes = 0);
// h and s of the hash-generated sketch with key `key` (see hash_word).
hipError_t launch_hash_sketch(int64_t d, int64_t k, uint64_t key, int32_t *h, int8_t *s,
                              hipStream_t st);
// Bytes of the optional per-die partial buffer of launch_cs_lds (0 when the
// per-die partial schedule does not pay for this shape); wd = element bytes.
size_t cs_part_bytes(int64_t d, int64_t k, int64_t ncols, int64_t wd);
template <typename T>
hipError_t launch_cs_sorted(int64_t k, const Cols<T> &c, const int32_t *off,
                            const uint32_t *sperm, T *Y, int64_t ldy, hipStream_t st);

// gemm.hip -- Z = G Y through split-K partial sums reduced in a fixed order.
struct GemmPlan {
  int M, N;
  int64_t K;
  int tiles_m, tiles_n, nsplit;
  int64_t kchunk;
  size_t partial_bytes;  // workspace for the split-K partials
  size_t ybf16_bytes;    // workspace for the BF16 copy of Y (BF16 path)
};
GemmPlan plan_gemm(int64_t M, int64_t N, int64_t K, ms_dtype g_dtype);
// z64 (optional) receives an FP64 copy of Z (ldz64 = M).
// yterms: for a BF16 G, Y enters as 1 BF16 term (rounded) or as 3 BF16
// terms whose sum is Y exactly.
hipError_t launch_gemm(const GemmPlan &p, ms_dtype g_dtype, const void *G, int64_t ldg,
                       const void *Y, int64_t ldy, void *Z, int64_t ldz, double *z64,
                       void *partials, void *ybf16, hipStream_t st, int yterms = 1);

// Z64 (M x N, ld M) = G Y64 in FP64 for N <= 8 (refinement correction).
size_t gemv64_partial_bytes(int64_t M, int64_t N, int64_t K);
hipError_t launch_gemv64(int64_t M, int64_t N, int64_t K, ms_dtype g_dtype, const void *G,
                         int64_t ldg, const double *Y, int64_t ldy, double *z64, double *part,
                         hipStream_t st);

// qr.hip -- Householder QR least squares of a small FP64 system.
size_t qr_workspace_bytes(int64_t m, int64_t n, int64_t nrhs);
hipError_t launch_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W, int64_t ldw,
                           const double *Bm, int64_t ldb, double *X, int64_t ldx, double *R,
                           int64_t ldr, double *tau_out, double *fact_out, void *qr_ws,
                           int *status, hipStream_t st);
// Register-resident variant for small systems (m <= 256, n + nrhs <= 144,
// n (n + nrhs) doubles in LDS); input [W | Bm] or split-K partials (part: FP64,
// part32: FP32, summed in split order).  hipErrorNotSupported when it does
// not fit.
bool qr_reg_fits(int64_t m, int64_t n, int64_t nrhs);
hipError_t launch_qr_reg(int64_t m, int64_t n, int64_t nrhs, const double *W, int64_t ldw,
                         const double *Bm, int64_t ldb, const double *part, const float *part32,
                         int nsplit, double *X, int64_t ldx, double *R, int64_t ldr,
                         double *tau_out, double *fact_out, int *status, hipStream_t st);
// X = R^{-1} (Q^T Bm)_{0:n} from factors kept by launch_qr_solve (fact: m x n
// with R on and above the diagonal and the reflector tails below, ld m; tau:
// n).  Bm (m x nrhs, ld m) is overwritten.
hipError_t launch_qr_apply_solve(int64_t m, int64_t n, int64_t nrhs, const double *fact,
                                 const double *tau, double *Bm, double *X, int64_t ldx,
                                 int *status, hipStream_t st);

// rand_cholQR least squares (randcholqr.hip): R0^{-1} of the sketch's R
// factor, the fused pass Q0 = A R0^{-1} -> Q0^T [Q0 | B] (per-workgroup
// partials), then the ordered sum, Cholesky and the two triangular solves.
// With Rinv and R0 null the same kernels solve the normal equations
// (W = [A | B]^T [A | B], R = chol(A^T A)).
constexpr int kRcqMaxN = 64;     // columns of A
constexpr int kRcqMaxRhs = 16;   // right-hand sides
constexpr int kRcqMaxCols = 80;  // n + nrhs (the partial's row length)
size_t rcq_partial_bytes(int grid);
int rcq_grid();
hipError_t launch_rcq_trinv(int n, const double *R0, int ldr0, double *Rinv, int *status,
                            hipStream_t st);
template <typename TA>
hipError_t launch_rcq_gram(int64_t d, int n, int nrhs, const TA *A, int64_t lda, const TA *B,
                           int64_t ldb, const double *Rinv, double *part, int grid,
                           hipStream_t st);
hipError_t launch_rcq_finish(int n, int nrhs, int nparts, const double *part, double *W,
                             const double *R0, int ldr0, const double *Rinv, double *X,
                             int64_t ldx, double *R, int64_t ldr, int *status, hipStream_t st);

// SRHT (srht.hip): Y = k^{-1/2} P H_m D X for an mx x ncols X (FP64 or FP32),
// m = the smallest power of two >= mx; Y k x ncols FP64.  part: the
// per-block partials (srht_workspace_bytes; none when m <= 8192).
int64_t srht_padded_rows(int64_t mx);
size_t srht_workspace_bytes(int64_t mx, int64_t ncols, int64_t k);
template <typename TX>
hipError_t launch_srht(int64_t mx, int64_t ncols, int64_t k, const TX *X, int64_t ldx,
                       const int8_t *dsign, const int32_t *r, double *Y, int64_t ldy, void *part,
                       int *status, hipStream_t st);

// ---------------------------------------------------------------- batched
// Item order of a persistent grid that keeps runs of consecutive items on
// one die: workgroup g runs on die g % dies (the dispatcher's round-robin),
// and with w = grid / dies workgroups per die, item (r dies + die) w + q goes
// to the q-th workgroup of that die.  Items that share data sit next to each
// other in every item order here, so they are fetched through the same L2.
// dies = 1 (grid not a multiple of the die count) is the plain order.
struct DieOrder {
  int64_t dies, die, q, wpd;
  __device__ explicit DieOrder(int ndies)
      : dies(ndies), die(blockIdx.x % ndies), q(blockIdx.x / ndies), wpd(gridDim.x / ndies) {}
  __device__ int64_t item(int64_t r) const { return (r * dies + die) * wpd + q; }
};
// the die count for a persistent grid of `grid` workgroups
inline int grid_dies(int grid, int xcds) { return xcds > 0 && grid % xcds == 0 ? xcds : 1; }

// Per-problem plan of a batched call, computed identically on the host (to
// size the workspace) and on the device (so graph replays with rewritten
// descriptors need no host work).
struct BatchEntry {
  int64_t cs_start;    // first CountSketch work item of the problem
  int64_t gemm_start;  // first Gaussian-stage work item
  int64_t y_off;       // byte offsets into the Y / partials / Z areas
  int64_t part_off;
  int64_t z_off;
  int64_t rows;        // rows per CountSketch item
  int64_t kchunk;      // K per Gaussian-stage item
  int64_t ktile;       // buckets per LDS tile
  int64_t code_off;    // byte offset of the packed bucket/sign words (d x 4 bytes), or -1
  int32_t nc, nt, ntiles, nsegs, nbt, tiles_m, tiles_n, nsplit;
  int32_t valid, pad2, refine, pad0;
  // refinement (refine != 0): residual r = B - A X (FP64, d x nrhs), its
  // CountSketch Yr (k x nrhs, FP64), G Yr split-K partials, and the QR
  // factors (k2 x n reflectors and R, then n values of tau)
  int64_t res_start, rcs_start, gv_start;
  int64_t f_off, r_off, yr_off, gv_off;
  int64_t rktile;
  int32_t rnt, rntiles, rnbt, pad1;
  // deterministic mode (det != 0): the block-ordered CountSketch instead of
  // the LDS one -- sorted keys of each 4096-row block at key_off, fold items
  // (column, bucket part) of the first pass and of the residuals
  int64_t bk_start, bf_start, bfr_start, key_off;
  int32_t det, parts, rparts, pad3;
};

constexpr int64_t kBatchResRows = 2048;  // rows per residual work item
constexpr int kBatchMaxRefineRhs = 8;

constexpr int64_t kBatchLdsSlots = 16384;  // FP64 partial sums per workgroup (128 KB)
constexpr int kBatchMaxK2 = 256;
constexpr int kBatchMaxCols = 144;

__host__ __device__ inline int64_t batch_align(int64_t x) { return (x + 255) / 256 * 256; }

// Sizes of one problem's items and areas.  wdata: bytes of A; accw: bytes of
// a Gaussian-stage partial; rows_item, kchunk: tuning (powers of two).
// Buckets per LDS tile and columns per tile for a CountSketch of nc columns.
__host__ __device__ inline void batch_cs_geom(int64_t k, int nc, int64_t &ktile, int32_t &nbt,
                                              int32_t &nt, int32_t &ntiles) {
  ktile = k;
  if (ktile > kBatchLdsSlots) {
    ktile = 1;
    while (ktile * 2 <= kBatchLdsSlots) ktile *= 2;
  }
  nbt = (int32_t)((k + ktile - 1) / ktile);
  nt = 1;
  while (nt < 4 && ktile * nt * 2 <= kBatchLdsSlots && nt * 2 <= nc) nt *= 2;
  ntiles = (nc + nt - 1) / nt;
}

// Deterministic mode: rows per sorted-key block, and the bucket sums one
// 160 KB workgroup holds next to a block's staged values and keys (FP32 data:
// 32768, FP64 data and residuals: 14336).
constexpr int64_t kBatchBfRows = 4096;
constexpr int kBatchBfMaxParts = 32;
__host__ __device__ inline int64_t batch_bf_slots(int welem) {
  return welem == 4 ? 32768 : 14336;
}

// Output tile of the Gaussian stage's work items: 256 x 144 for a 16-bit G
// (the wide matrix-core tile of gemm.hip), 64 x 64 else.
constexpr int kBatchWideTM = 256, kBatchWideTN = 144;

__host__ __device__ inline void batch_entry(const ms_problem &P, int wdata, int accw,
                                            int64_t rows_item, int64_t kchunk, int refine,
                                            BatchEntry &E, int det = 0, int g16 = 0) {
  E = BatchEntry{};
  E.valid = P.d >= 1 && P.d < 0x7fffffffLL && P.n >= 1 && P.nrhs >= 1 && P.k >= 1 &&
            P.k < 0x7fffffffLL && P.k2 >= P.n && P.k2 <= kBatchMaxK2 &&
            P.n + P.nrhs <= kBatchMaxCols && P.lda >= P.d && P.ldb >= P.d && P.ldg >= P.k2 &&
            P.ldx >= P.n && P.A && P.B && P.h && P.s && P.G && P.X &&
            (!refine || P.nrhs <= kBatchMaxRefineRhs);
  if (!E.valid) return;
  E.nc = (int32_t)(P.n + P.nrhs);
  batch_cs_geom(P.k, E.nc, E.ktile, E.nbt, E.nt, E.ntiles);
  E.refine = refine ? 1 : 0;
  if (refine) batch_cs_geom(P.k, (int)P.nrhs, E.rktile, E.rnbt, E.rnt, E.rntiles);
  // rows per item: an item adds rows * ktile / k values into a tile of ktile
  // slots and flushes the tile once, so at least 8 k rows keep the flush
  // (global atomics) under an eighth of the adds
  E.rows = rows_item;
  while (E.rows < 8 * P.k && E.rows < ((int64_t)1 << 30)) E.rows *= 2;
  E.nsegs = (int32_t)((P.d + E.rows - 1) / E.rows);
  E.tiles_m = (int32_t)(g16 ? (P.k2 + kBatchWideTM - 1) / kBatchWideTM : (P.k2 + 63) / 64);
  E.tiles_n = g16 ? (E.nc + kBatchWideTN - 1) / kBatchWideTN : (E.nc + 63) / 64;
  E.kchunk = kchunk;
  E.nsplit = (int32_t)((P.k + kchunk - 1) / kchunk);
  if (det) {
    E.det = 1;
    const int64_t parts = (P.k + batch_bf_slots(wdata) - 1) / batch_bf_slots(wdata);
    const int64_t rparts = (P.k + batch_bf_slots(8) - 1) / batch_bf_slots(8);
    if (parts > kBatchBfMaxParts || rparts > kBatchBfMaxParts || P.k >= ((int64_t)1 << 19)) {
      E.valid = 0;
      return;
    }
    E.parts = (int32_t)parts;
    E.rparts = refine ? (int32_t)rparts : 0;
  }
}

__host__ __device__ inline int64_t batch_cs_items(const BatchEntry &E) {
  return E.valid && !E.det ? (int64_t)E.ntiles * E.nsegs * E.nbt : 0;
}
// deterministic mode: key blocks, fold items, key bytes
__host__ __device__ inline int64_t batch_bk_items(const ms_problem &P, const BatchEntry &E) {
  return E.valid && E.det ? (P.d + kBatchBfRows - 1) / kBatchBfRows : 0;
}
__host__ __device__ inline int64_t batch_bf_items(const BatchEntry &E) {
  return E.valid && E.det ? (int64_t)E.nc * E.parts : 0;
}
__host__ __device__ inline int64_t batch_bfr_items(const ms_problem &P, const BatchEntry &E) {
  return E.valid && E.det && E.refine ? (int64_t)P.nrhs * E.rparts : 0;
}
__host__ __device__ inline int64_t batch_key_bytes(const ms_problem &P, const BatchEntry &E) {
  return batch_bk_items(P, E) * kBatchBfRows * 4;
}
__host__ __device__ inline int64_t batch_gemm_items(const BatchEntry &E) {
  return E.valid ? (int64_t)E.tiles_m * E.tiles_n * E.nsplit : 0;
}
__host__ __device__ inline int64_t batch_y_bytes(const ms_problem &P, const BatchEntry &E, int wdata) {
  return E.valid ? batch_align(P.k * E.nc * wdata) : 0;
}
// Rows are packed into bucket/sign words only when the CountSketch sweeps
// them at least kBatchPackSweeps times (column tiles x bucket tiles): the
// pack pass (9 bytes per row) pays for itself from there.
constexpr int kBatchPackSweeps = 8;
__host__ __device__ inline bool batch_packs(const BatchEntry &E) {
  return E.valid && !E.det && (int64_t)E.ntiles * E.nbt >= kBatchPackSweeps;
}
__host__ __device__ inline int64_t batch_code_bytes(const ms_problem &P, const BatchEntry &E) {
  return batch_packs(E) ? batch_align(P.d * 4) : 0;
}
__host__ __device__ inline int64_t batch_part_bytes(const ms_problem &P, const BatchEntry &E, int accw) {
  return E.valid ? batch_align((int64_t)E.nsplit * P.k2 * E.nc * accw) : 0;
}
__host__ __device__ inline int64_t batch_z_bytes(const ms_problem &P, const BatchEntry &E) {
  return E.valid ? batch_align(P.k2 * E.nc * 8) : 0;
}
// refinement items and areas (zero without refinement)
__host__ __device__ inline bool batch_ref(const BatchEntry &E) { return E.valid && E.refine; }
__host__ __device__ inline int64_t batch_res_items(const ms_problem &P, const BatchEntry &E) {
  return batch_ref(E) ? (P.d + kBatchResRows - 1) / kBatchResRows : 0;
}
__host__ __device__ inline int64_t batch_rcs_items(const BatchEntry &E) {
  return batch_ref(E) && !E.det ? (int64_t)E.rntiles * E.nsegs * E.rnbt : 0;
}
__host__ __device__ inline int64_t batch_gv_items(const BatchEntry &E) {
  return batch_ref(E) ? (int64_t)E.nsplit : 0;
}
__host__ __device__ inline int64_t batch_f_bytes(const ms_problem &P, const BatchEntry &E) {
  return batch_ref(E) ? batch_align((P.k2 * P.n + P.n) * 8) : 0;
}
__host__ __device__ inline int64_t batch_r_bytes(const ms_problem &P, const BatchEntry &E) {
  return batch_ref(E) ? batch_align(P.d * P.nrhs * 8) : 0;
}
__host__ __device__ inline int64_t batch_yr_bytes(const ms_problem &P, const BatchEntry &E) {
  return batch_ref(E) ? batch_align(P.k * P.nrhs * 8) : 0;
}
__host__ __device__ inline int64_t batch_gv_bytes(const ms_problem &P, const BatchEntry &E) {
  return batch_ref(E) ? batch_align((int64_t)E.nsplit * P.k2 * P.nrhs * 8) : 0;
}

// Totals written by the setup kernel (device) next to the entries.
struct BatchTotals {
  int64_t cs_items, gemm_items, y_bytes, part_bytes, z_bytes, max_mn;
  int64_t res_items, rcs_items, gv_items, yr_bytes;
  int64_t bk_items, bf_items, bfr_items;
  int64_t pad[3];
};

// Last problem whose first item (member M of its entry) is <= it; problems
// without items share the next problem's start and so are never selected.
template <int64_t BatchEntry::*M>
__device__ __forceinline__ int batch_find_m(const BatchEntry *__restrict__ E, int count,
                                            int64_t it) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (E[mid].*M <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// countsketch.hip / gemm.hip / qr.hip batched launchers
// packed words h | sign << 31 of every problem's rows into the code area
// (invalid rows: 0xffffffff and MS_ERR_RANGE for the problem)
hipError_t launch_batch_pack(int count, const ms_problem *P, const BatchEntry *E,
                             unsigned char *codearea, int *pstatus, int *status, hipStream_t st);
template <typename T>
hipError_t launch_batch_cs(int count, const ms_problem *P, const BatchEntry *E,
                           const BatchTotals *tot, const unsigned char *codearea,
                           unsigned char *yarea, int *pstatus, int *status, int grid,
                           hipStream_t st);
hipError_t launch_batch_gemm(int count, ms_dtype g_dtype, const ms_problem *P,
                             const BatchEntry *E, const BatchTotals *tot,
                             const unsigned char *yarea, unsigned char *parea, int grid,
                             hipStream_t st, int yterms = 1);
hipError_t launch_batch_reduce(int count, ms_dtype g_dtype, const ms_problem *P,
                               const BatchEntry *E, const unsigned char *parea,
                               unsigned char *zarea, int max_mn, hipStream_t st);
hipError_t launch_batch_qr(int count, int max_k2, int max_n, int max_nc, const ms_problem *P,
                           const BatchEntry *E, const unsigned char *zarea, unsigned char *farea,
                           int *pstatus, int *status, hipStream_t st,
                           int det = 0);
// refinement: r = B - A X; Yr = C r; partials of G Yr; X += R^{-1} Q^T (G Yr)
template <typename TA>
hipError_t launch_batch_residual(int count, const ms_problem *P, const BatchEntry *E,
                                 const BatchTotals *tot, unsigned char *rarea, int grid,
                                 hipStream_t st);
hipError_t launch_batch_cs_res(int count, const ms_problem *P, const BatchEntry *E,
                               const BatchTotals *tot, const unsigned char *codearea,
                               const unsigned char *rarea, unsigned char *yrarea, int *pstatus,
                               int *status, int grid, hipStream_t st);
hipError_t launch_batch_gemv(int count, ms_dtype g_dtype, const ms_problem *P,
                             const BatchEntry *E, const BatchTotals *tot,
                             const unsigned char *yrarea, unsigned char *gvarea, int grid,
                             hipStream_t st);
// tol_log2 > 0: a problem whose correction is <= 2^-tol_log2 of its X
// (Frobenius) has its entry's refine flag cleared, and the later steps'
// residual, sketch, G product and update kernels skip it
hipError_t launch_batch_apply_solve(int count, const ms_problem *P, BatchEntry *E,
                                    const unsigned char *gvarea, const unsigned char *farea,
                                    int *pstatus, int *status, hipStream_t st, int tol_log2 = 0);

// ------------------------------------------------------------------ wave helpers
// Wave-wide sum with DPP: quad swaps, half-row and row mirrors give every
// lane its 16-lane row sum, two row broadcasts (lane 15 into rows 1 and 3,
// lane 31 into rows 2 and 3) leave the total in lane 63, and one lane read
// (a pair, for the two halves of the double) hands it to every lane.
// Every lane is written (all rows and banks enabled, and each of these
// patterns reads a lane of its own row), so the move needs no prior value and
// no zeroed destination register.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long u = __double_as_longlong(v);
  int lo = (int)(u & 0xffffffffLL), hi = (int)(u >> 32);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// DPP broadcast into the rows selected by ROWMASK; other rows get 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_bcast(double v) {
  const long long u = __double_as_longlong(v);
  int lo = (int)(u & 0xffffffffLL), hi = (int)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_allsum(double v) {
  v += dpp_move<0xb1>(v);        // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);        // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);       // row_half_mirror
  v += dpp_move<0x140>(v);       // row_mirror: every lane holds its 16-lane row sum
  v += dpp_bcast<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3: rows (0+1), (2+3)
  v += dpp_bcast<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3: lane 63 holds the total
  return read_lane(v, 63);
}

// Ascending sort of 4096 32-bit keys by their low 31 bits (bit 31 is carried
// along; keys whose low bits are equal must be equal in full, as the padding
// keys are), by the 1024 threads of a workgroup: a bitonic network run on four
// keys per thread in registers, thread t holding positions 4t .. 4t + 3 in v
// on entry and on return.  Strides 1 and 2 stay inside a thread, strides 4 to
// 128 are exchanges between the lanes of one wave (a wave holds 256
// consecutive keys), and only strides of 256 and more go through the LDS
// scratch key (4096 keys, 16-byte aligned), one barrier each.  Every thread
// reads back only its own positions after the last barrier, so the scratch
// may be rewritten (own positions first) without another barrier.
__device__ __forceinline__ void sort4096_regs(uint32_t (&v)[4], uint32_t *key) {
  constexpr uint32_t M = 0x7fffffffu;
  const int t = threadIdx.x;
  for (int size = 2; size <= 4096; size <<= 1) {
    int stride = size >> 1;
    if (stride >= 256) {
      // each thread stores and later reloads only its own four positions, so
      // the previous phase needs no barrier before the store
      *reinterpret_cast<uint4 *>(key + 4 * t) = make_uint4(v[0], v[1], v[2], v[3]);
      __syncthreads();
      for (; stride >= 256; stride >>= 1) {
        for (int u = t; u < 2048; u += 1024) {
          const int lo = 2 * u - (u & (stride - 1));
          const int hi = lo + stride;
          const bool up = (lo & size) == 0;
          const uint32_t x = key[lo], y = key[hi];
          if (((x & M) > (y & M)) == up) {
            key[lo] = y;
            key[hi] = x;
          }
        }
        __syncthreads();
      }
      const uint4 q = *reinterpret_cast<const uint4 *>(key + 4 * t);
      v[0] = q.x;
      v[1] = q.y;
      v[2] = q.z;
      v[3] = q.w;
    }
    for (; stride >= 4; stride >>= 1) {
      const int lm = stride >> 2;   // partner thread t ^ lm, in the same wave
      const bool lower = (t & lm) == 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool up = ((4 * t + i) & size) == 0;
        const uint32_t o = (uint32_t)__shfl_xor((int)v[i], lm, 64);
        const bool o_less = (o & M) < (v[i] & M), v_less = (v[i] & M) < (o & M);
        v[i] = lower == up ? (o_less ? o : v[i]) : (v_less ? o : v[i]);
      }
    }
    for (; stride >= 1; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i & stride) continue;
        const int j = i | stride;
        const bool up = ((4 * t + i) & size) == 0;
        if (((v[i] & M) > (v[j] & M)) == up) {
          const uint32_t x = v[i];
          v[i] = v[j];
          v[j] = x;
        }
      }
    }
  }
}
// The same sort of the 4096 keys held in key (LDS, 16-byte aligned): enter
// with the workgroup synchronised on key; on return the sorted keys are in
// key and the workgroup is synchronised.
__device__ __forceinline__ void sort4096_lds(uint32_t *key) {
  const int t = threadIdx.x;
  const uint4 q = *reinterpret_cast<const uint4 *>(key + 4 * t);
  uint32_t v[4] = {q.x, q.y, q.z, q.w};
  sort4096_regs(v, key);
  *reinterpret_cast<uint4 *>(key + 4 * t) = make_uint4(v[0], v[1], v[2], v[3]);
  __syncthreads();
}

// cs_tiled.hip -- the CountSketch for bucket counts beyond one workgroup's
// LDS (k > 16384): a per-call plan grouping each 8192-row block's rows by
// bucket tile, then one pass in which each tile's workgroups visit only
// their own rows.
// Bytes of the plan (0 when the tiled CountSketch does not apply to d, k).
size_t cs_tile_plan_bytes(int64_t d, int64_t k);
// The current device can run the tiled CountSketch for (d, k).
bool cs_tiled_supported(int64_t d, int64_t k);
// Build the plan from packed codes (code non-null) or from h and s (checked:
// MS_ERR_RANGE for a bad row, which the plan then leaves out).
hipError_t launch_tile_plan(int64_t d, int64_t k, const uint32_t *code, const int32_t *h,
                            const int8_t *s, void *plan, int *status, hipStream_t st);
// Y += C [A | B] from the plan (Y is not cleared).
template <typename T>
hipError_t launch_cs_tiled(int64_t d, int64_t k, const Cols<T> &c, const void *plan, T *Y,
                           int64_t ldy, hipStream_t st);

// ne_wide.hip -- the normal equations / rand_cholQR's Cholesky stage for
// wide problems (n <= 256, nrhs <= 16, n + nrhs <= 272): the Gram product
// W = [X | B]^T [X | B] of a tall V in FP64 (per-chunk partials of upper
// tiles, summed in chunk order), then R1 = chol(W_XX), y = R1^{-T} W_XB,
// x = R1^{-1} y (and x = R0^{-1} x when fact holds rand_cholQR's R0).
constexpr int kWideMaxN = 256;
constexpr int kWideMaxRhs = 16;
constexpr int kWideMaxCols = 272;
int gram_wide_chunks(int64_t d, int nc);
size_t gram_wide_partial_bytes(int64_t d, int nc);
size_t gram_wide_w_bytes(int nc);
template <typename TX, typename TB>
hipError_t launch_gram_wide(int64_t d, int nx, int nc, const TX *X, int64_t ldx, const TB *B,
                            int64_t ldb, double *part, double *W, hipStream_t st);
// rand_cholQR for wide problems (rcq_wide.hip): Rinv (n x n, ld n) = R0^{-1}
// from the upper part of the QR factors (ld ldf), then Q0 = A Rinv (d x n
// FP64, ld d).  A zero or non-finite diagonal of R0 records MS_ERR_SINGULAR.
hipError_t launch_rcq_wide_q0(int64_t d, int n, ms_dtype a_dtype, const void *A, int64_t lda,
                              const double *fact, int64_t ldf, double *Rinv, double *Q0,
                              int *status, hipStream_t st);
// bad: one int of workspace (breakdown flag between the launches)
hipError_t launch_chol_solve_wide(int n, int nrhs, int nc, double *W, const double *fact,
                                  int64_t ldf, double *X, int64_t ldx, double *R, int64_t ldr,
                                  int *bad, int *status, hipStream_t st);

// plan_blocked.hip -- the sketch plan by 4096-row blocks with LDS counts (k <=
// 16384; no global atomics, stable without a per-bucket sort), and the
// deterministic fold launched a few columns at a time.
// Bytes of the blocks x k count table (0 when the blocked plan does not apply).
size_t plan_blocked_bytes(int64_t d, int64_t k);
hipError_t launch_plan_blocked(int64_t d, int64_t k, const int32_t *h, const int8_t *s,
                               int32_t *cnt, int32_t *off, int32_t *cursor, void *tab_ws,
                               uint32_t *sperm, int *status, hipStream_t st);
template <typename T>
hipError_t launch_cs_sorted_cols(int64_t k, const Cols<T> &c, const int32_t *off,
                                 const uint32_t *sperm, T *Y, int64_t ldy, hipStream_t st);

// deterministic batched mode (cs_blockfold.hip): sorted keys of every
// problem's 4096-row blocks; the block-ordered fold of every problem's
// [A | B] (RES = 0, into the Y area) or of its residuals (RES = 1, into Yr)
hipError_t launch_batch_bf_keys(int count, const ms_problem *P, const BatchEntry *E,
                                const BatchTotals *tot, unsigned char *keyarea, int *pstatus,
                                int *status, int grid, hipStream_t st);
template <typename T, int RES>
hipError_t launch_batch_bf_fold(int count, const ms_problem *P, const BatchEntry *E,
                                const BatchTotals *tot, const unsigned char *keyarea,
                                const unsigned char *rarea, unsigned char *out, int grid,
                                hipStream_t st);

// cs_blockfold.hip -- the deterministic CountSketch as a block-ordered fold:
// per block of 4096 rows the keys (bucket << 12 | row | sign << 31) sorted
// by (bucket, row); then one workgroup per (column, bucket range) folds the
// blocks in order with its bucket sums in LDS (elem: bytes of the data type).
bool cs_blockfold_supported(int64_t d, int64_t k, int ncols, size_t elem);
size_t cs_blockfold_key_bytes(int64_t d);
hipError_t launch_bf_keys(int64_t d, int64_t k, const int32_t *h, const int8_t *s, uint32_t *keys,
                          int *status, hipStream_t st);
template <typename T>
hipError_t launch_bf_fold(int64_t d, int64_t k, const Cols<T> &c, const uint32_t *keys, T *Y,
                          int64_t ldy, hipStream_t st);

}  // namespace ms
