// randcholqr.hip -- rand_cholQR least squares (Alg. 5, Sec. 6.3) after the
// multisketch: given R0 (the R factor of the sketched A, from the register
// QR), form Q0 = A R0^{-1}, the Gram matrix Q0^T Q0 and Q0^T B in one pass
// over A and B, then R1 = chol(Q0^T Q0), R = R1 R0, y = R1^{-T} Q0^T B and
// x = R^{-1} y.  The result is the least-squares optimum of min ||B - A x||:
// the sketch only preconditions.  Without R0 the same kernels solve the
// normal equations (Sec. 6.3's comparator).
//
// The pass over A is the dominant cost (n(n+1) flops per row for Q0 and as
// many for the upper Gram matrix, FP64): persistent workgroups of eight
// waves; each wave takes 16-row slabs, forms the slab's Q0 tiles on the f64
// matrix cores (R0^{-1} staged in LDS, its zero lower blocks skipped) and
// accumulates the upper tiles of Q0^T [Q0 | B] straight from those result
// registers (see k_rcq_gram).  Q0 never leaves the registers: A and B are
// read once.  The waves' and then the workgroups' partial products are
// summed in a fixed order, then one wave factors and solves.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
// four consecutive elements at element alignment (a dword-aligned multi-dword
// global load is legal)
typedef double dvec4e __attribute__((ext_vector_type(4), aligned(8)));
typedef float fvec4e __attribute__((ext_vector_type(4), aligned(4)));
template <typename T>
struct Four;
template <>
struct Four<double> {
  typedef dvec4e type;
};
template <>
struct Four<float> {
  typedef fvec4e type;
};

// Rows row .. row + 3 of the column at p (all inside the column), FP64.
template <typename T>
__device__ __forceinline__ v4d load_rows4_full(const T *p, int64_t row) {
  const typename Four<T>::type x = gload((const typename Four<T>::type *)(p + row));
  return v4d{(double)x[0], (double)x[1], (double)x[2], (double)x[3]};
}

// Rows row .. row + 3 of the column at p (zero past row d, or for p null),
// promoted to FP64.
template <typename T>
__device__ __forceinline__ v4d load_rows4(const T *p, int64_t row, int64_t d) {
  v4d v = v4d{0.0, 0.0, 0.0, 0.0};
  if (p == nullptr) return v;
  if (row + 4 <= d) {
    const typename Four<T>::type x = gload((const typename Four<T>::type *)(p + row));
    v = v4d{(double)x[0], (double)x[1], (double)x[2], (double)x[3]};
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (row + r < d) v[r] = (double)gload(p + row + r);
  }
  return v;
}

constexpr int kLdr = 68;   // LDS row stride of R0^{-1} (doubles)
constexpr int kPart = kRcqMaxN * kRcqMaxCols;  // doubles of one partial (64 x 80, row-major)

__device__ __forceinline__ v4d mma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// R0^{-1} (64 x 64, row-major, zero outside the leading n x n block) by
// back substitution, R0 x = e_j for every column j, on four waves: wave w
// takes columns 16 w .. 16 w + 15 (lane & 15), and the four 16-lane groups
// g = lane >> 4 of a wave split each step's sum by row residue:
//   x_i = (delta_ij - sum_{l > i} R0[i][l] x_l) / R0[i][i],
// group g adding the terms l = g (mod 4) from its 16 registers
// (x[m] = x_{4m+g}), two xor shuffles giving every group the whole sum.  A
// wave skips the steps below its columns' rows (x_i = 0 for i > j).
__global__ __launch_bounds__(256) void k_rcq_trinv(int n, const double *__restrict__ R0, int ldr0,
                                                   double *__restrict__ Rinv, int *status) {
  constexpr int N = kRcqMaxN, L = kRcqMaxN + 1;
  __shared__ double r0[N * L];  // row-major: r0[i L + l] = R0[i][l], zero elsewhere
  __shared__ double dinv[N];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int t = tid; t < N * N; t += 256) {
    const int i = t & (N - 1), l = t >> 6;  // coalesced along the column
    r0[i * L + l] = (i < n && l < n && i <= l) ? R0[i + (int64_t)l * ldr0] : 0.0;
  }
  if (tid < N) {
    const double dii = tid < n ? R0[tid + (int64_t)tid * ldr0] : 1.0;
    const bool bad = tid < n && (!(dii != 0.0) || !isfinite(dii));
    dinv[tid] = tid < n ? 1.0 / dii : 0.0;
    if (__any(bad) && tid == 0) record_status(status, MS_ERR_SINGULAR);
  }
  __syncthreads();
  const int j = 16 * w + (lane & 15), g = lane >> 4;
  double x[N / 4];
#pragma unroll
  for (int m = 0; m < N / 4; ++m) x[m] = 0.0;
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    if (i > 16 * w + 15) continue;  // wave-uniform: every column of this wave is left of row i
    double acc[2] = {0.0, 0.0};
    // terms l = 4 m + g > i; entries at l <= i are zero (r0's lower part, or
    // the not yet computed x_i), so the static range may start early
#pragma unroll
    for (int m = (i + 1) / 4 > 0 ? ((i + 1) / 4 - 1 > 0 ? (i + 1) / 4 - 1 : 0) : 0; m < N / 4; ++m)
      acc[m & 1] += r0[i * L + 4 * m + g] * x[m];
    double sum = acc[0] + acc[1];
    sum += __shfl_xor(sum, 16);
    sum += __shfl_xor(sum, 32);
    const double xi = ((i == j) ? 1.0 : 0.0) - sum;
    if (g == (i & 3)) x[i >> 2] = xi * dinv[i];
  }
#pragma unroll
  for (int m = 0; m < N / 4; ++m) Rinv[(4 * m + g) * N + j] = x[m];
}

// The fused pass.  NTI = column tiles of Q0 (n <= 16 NTI).  The columns of
// B that do not fit in Q0's last tile (nx = n + nrhs - 16 NTI of them) are
// handled by EXTRA: 0 (none), 1 (one more 16-column MFMA tile), 2 (nx = 1:
// vector FMAs, since a tile with one column in use would cost 4 NTI
// matrix-core instructions per slab).  PLAIN: no R0 (the normal equations,
// Sec. 6.3): V = [A | B] itself, W = V^T V.
//
// Each wave takes slabs of 16 rows of A (grid-stride over all waves).  For a
// slab it forms the 16 x 16 NTI block of Q0 = A R0^{-1} on the f64 matrix
// cores: the A operand of k-step ks is A[row li][4 ks + lk] (lane li + 16 lk),
// the B operand R0^{-1}[4 ks + lk][16 jt + li] from LDS, and the result
// register r of column tile jt is Q0[lk + 4 r][16 jt + li].  That is exactly
// the operand layout of the Gram products over the slab's 16 rows
// (k = row): A operand Q0[4 r + lk][16 it + li], B operand
// V[4 r + lk][16 ct + li] with V = [Q0 | B], so the tiles (it, ct), it <= ct,
// of V^T V accumulate from registers with no data exchange between lanes.
// B's columns enter V's tiles from the lanes whose column is >= n (R0^{-1}
// is zero there, so those lanes' Q0 values are zero).  After its last slab
// each wave holds the sum over its slabs; the waves are added in wave order
// through LDS and the workgroup's partial (row-major 64 x 80: entry (i, j) at
// i 80 + j; upper tiles only) goes to part[blockIdx.x].  Eight waves (two per
// SIMD) keep the matrix cores busy while a wave waits for its slab.
//
// In the PLAIN form the operands come from memory directly: the Gram
// product only needs both operands to map the k index to the same row, so
// lane (li, lk) takes rows 4 lk .. 4 lk + 3 of column 16 ct + li with one
// vector load (register r = row 4 lk + r).
constexpr int kGramWaves = 8;
template <typename TA, int NTI, int EXTRA, bool PLAIN>
__global__ __launch_bounds__(64 * kGramWaves) void k_rcq_gram(int64_t d, int n, int nrhs,
                                                              const TA *__restrict__ A,
                                                              int64_t lda,
                                                              const TA *__restrict__ B,
                                                              int64_t ldb,
                                                              const double *__restrict__ Rinv,
                                                              double *__restrict__ part) {
  constexpr int NCT = NTI + (EXTRA == 1);
  constexpr int NT = NTI * NCT - NTI * (NTI - 1) / 2;  // tiles (it, ct), it <= ct
  constexpr int NZ = EXTRA == 2 ? 1 : 0;                // vector columns of B
  constexpr int NB = EXTRA == 1 ? 2 : 1;                // B fragments in MFMA tiles
  __shared__ double rinv[kRcqMaxN * kLdr];             // rinv[k kLdr + j] = R0^{-1}[k][j]
  __shared__ double wsum[kRcqMaxN * kRcqMaxCols];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  if (!PLAIN) {
    for (int t = tid; t < kRcqMaxN * kRcqMaxN; t += 64 * kGramWaves)
      rinv[(t >> 6) * kLdr + (t & 63)] = Rinv[t];
    __syncthreads();
  }

  v4d w[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) w[u] = v4d{0.0, 0.0, 0.0, 0.0};
  double z[NTI][NZ > 0 ? NZ : 1];
#pragma unroll
  for (int it = 0; it < NTI; ++it)
#pragma unroll
    for (int c = 0; c < (NZ > 0 ? NZ : 1); ++c) z[it][c] = 0.0;
  const int zc0 = 16 * NTI - n;                  // first B column outside Q0's tiles
  const int nx = EXTRA == 2 ? nrhs - zc0 : 0;    // vector columns in use

  const int64_t nslab = (d + 15) >> 4;
  const int64_t stride = (int64_t)gridDim.x * kGramWaves;
  // per-lane bases; the per-k-step offsets 4 ks lda are wave-uniform
  const TA *const Al = A + li + (int64_t)lk * lda;
  const int64_t lda4 = 4 * lda;
  // PLAIN: the column each lane reads in tile ct (A's, B's, or none)
  const TA *vcol[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int c = 16 * ct + li;
    vcol[ct] = c < n ? A + (int64_t)c * lda : (c - n < nrhs ? B + (int64_t)(c - n) * ldb : nullptr);
  }
  const TA *const zcol = NZ > 0 ? B + (int64_t)zc0 * ldb : nullptr;
  // Full slabs (all 16 rows inside A) load without any branch: a load
  // behind a per-lane branch is waited for at the branch's end, which
  // serialises the slab's loads.  A lane without a column reads A's first
  // column and masks the value; only the last, ragged slab takes the
  // guarded path.
  const int64_t nfull = d >> 4;
  // full slabs: the next slab's operands are loaded into registers while the
  // current one is multiplied (one slab ahead)
  v4d qn[NCT], zn = v4d{0.0, 0.0, 0.0, 0.0};
  auto load_full = [&](int64_t sl_) {
    const int64_t rr_ = sl_ * 16 + 4 * lk;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) qn[ct] = load_rows4_full(vcol[ct] ? vcol[ct] : A, rr_);
    if (NZ > 0) zn = load_rows4_full(zcol, rr_);
  };
  {
    const int64_t sl0 = (int64_t)blockIdx.x * kGramWaves + wave;
    if (PLAIN && sl0 < nfull) load_full(sl0);
  }
  for (int64_t sl = (int64_t)blockIdx.x * kGramWaves + wave; PLAIN && sl < nslab; sl += stride) {
    const int64_t rr = sl * 16 + 4 * lk;
    v4d q[NCT];
    v4d zb = v4d{0.0, 0.0, 0.0, 0.0};
    if (sl < nfull) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) q[ct] = qn[ct];
      if (NZ > 0) zb = zn;
      if (sl + stride < nfull) load_full(sl + stride);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
        if (!vcol[ct]) q[ct] = v4d{0.0, 0.0, 0.0, 0.0};
      if (NZ > 0 && nx <= 0) zb = v4d{0.0, 0.0, 0.0, 0.0};
    } else {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) q[ct] = load_rows4(vcol[ct], rr, d);
      if (NZ > 0 && nx > 0) zb = load_rows4(zcol, rr, d);
    }
    int u = 0;
#pragma unroll
    for (int it = 0; it < NTI; ++it)
#pragma unroll
      for (int ct = it; ct < NCT; ++ct, ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) w[u] = mma64(q[it][r], q[ct][r], w[u]);
    if (NZ > 0)
#pragma unroll
      for (int it = 0; it < NTI; ++it)
#pragma unroll
        for (int r = 0; r < 4; ++r) z[it][0] += q[it][r] * zb[r];
  }
  // B columns of this lane in the tiles NTI - 1 .. (clamped into [0, nrhs))
  const TA *fbcol[NB];
  bool fbok[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int c = 16 * (NTI - 1 + e) + li - n;
    fbok[e] = c >= 0 && c < nrhs;
    fbcol[e] = B + (int64_t)(c < 0 ? 0 : (c < nrhs ? c : nrhs - 1)) * ldb;
  }
  for (int64_t sl = (int64_t)blockIdx.x * kGramWaves + wave; !PLAIN && sl < nslab; sl += stride) {
    const int64_t r0 = sl * 16;
    double a[4 * NTI];
    // fb[e][r] = B[r0 + lk + 4 r][c], c = 16 (NTI - 1 + e) + li - n (zero
    // outside 0 <= c < nrhs); zb[c][r] = B[r0 + lk + 4 r][zc0 + c]
    double fb[NB][4];
    double zb[NZ > 0 ? NZ : 1][4];
    if (sl < nfull) {
      // no branch around any load (see the PLAIN loop): columns past n read
      // column n - 1 and B columns outside [0, nrhs) read a clamped one, and
      // the values are masked afterwards
#pragma unroll
      for (int ks = 0; ks < 4 * NTI; ++ks) {
        const int kk = 4 * ks + lk;
        a[ks] = (double)gload(A + li + r0 + (int64_t)min(kk, n - 1) * lda);
      }
#pragma unroll
      for (int e = 0; e < NB; ++e)
#pragma unroll
        for (int r = 0; r < 4; ++r) fb[e][r] = (double)gload(fbcol[e] + r0 + lk + 4 * r);
#pragma unroll
      for (int c = 0; c < NZ; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) zb[c][r] = (double)gload(zcol + r0 + lk + 4 * r);
#pragma unroll
      for (int ks = 0; ks < 4 * NTI; ++ks)
        if (4 * ks + lk >= n) a[ks] = 0.0;
#pragma unroll
      for (int e = 0; e < NB; ++e)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (!fbok[e]) fb[e][r] = 0.0;
#pragma unroll
      for (int c = 0; c < NZ; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (c >= nx) zb[c][r] = 0.0;
    } else {
      const bool rin = r0 + li < d;
      const TA *const As = Al + r0;
#pragma unroll
      for (int ks = 0; ks < 4 * NTI; ++ks)
        a[ks] = (rin && 4 * ks + lk < n) ? (double)gload(As + ks * lda4) : 0.0;
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int c = 16 * (NTI - 1 + e) + li - n;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t rw = r0 + lk + 4 * r;
          fb[e][r] = (c >= 0 && c < nrhs && rw < d) ? (double)gload(B + rw + (int64_t)c * ldb) : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < NZ; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t rw = r0 + lk + 4 * r;
          zb[c][r] = (c < nx && rw < d) ? (double)gload(B + rw + (int64_t)(zc0 + c) * ldb) : 0.0;
        }
    }
    // R0^{-1} is re-read from LDS in every slab: the empty asm keeps the
    // compiler from hoisting its 4 NTI (NTI + 1) / 2 fragments into registers
    // for the whole loop (which would leave too few for two waves per SIMD)
    int roff = lk * kLdr + li;
    asm volatile("" : "+v"(roff));
    v4d q[NCT];
#pragma unroll
    for (int jt = 0; jt < NCT; ++jt) q[jt] = v4d{0.0, 0.0, 0.0, 0.0};
    // Q0 tile jt: R0^{-1} is upper triangular, so k-step ks enters the tiles
    // jt >= ks / 4 only (k-step outer: each A fragment is used, then dead)
#pragma unroll
    for (int ks = 0; ks < 4 * NTI; ++ks)
#pragma unroll
      for (int jt = ks / 4; jt < NTI; ++jt)
        q[jt] = mma64(a[ks], rinv[roff + 4 * ks * kLdr + 16 * jt], q[jt]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      q[NTI - 1][r] += fb[0][r];
      if (EXTRA == 1) q[NCT - 1][r] = fb[NB - 1][r];
    }
    int u = 0;
#pragma unroll
    for (int it = 0; it < NTI; ++it)
#pragma unroll
      for (int ct = it; ct < NCT; ++ct, ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) w[u] = mma64(q[it][r], q[ct][r], w[u]);
    // vector columns: z[it][c] += sum_r Q0[lk + 4 r][16 it + li] B[lk + 4 r][zc0 + c]
#pragma unroll
    for (int c = 0; c < NZ; ++c)
      if (c < nx)
#pragma unroll
        for (int it = 0; it < NTI; ++it)
#pragma unroll
          for (int r = 0; r < 4; ++r) z[it][c] += q[it][r] * zb[c][r];
  }
  // vector columns: sum over the four lane rows lk (xor 16, then xor 32)
#pragma unroll
  for (int c = 0; c < NZ; ++c)
#pragma unroll
    for (int it = 0; it < NTI; ++it) {
      z[it][c] += __shfl_xor(z[it][c], 16);
      z[it][c] += __shfl_xor(z[it][c], 32);
    }
  // the waves' sums, added in wave order
  double *P = part + (int64_t)blockIdx.x * kPart;
  for (int wv = 0; wv < kGramWaves; ++wv) {
    if (wave == wv) {
      const bool first = wv == 0, last = wv == kGramWaves - 1;
      int u = 0;
#pragma unroll
      for (int it = 0; it < NTI; ++it)
#pragma unroll
        for (int ct = it; ct < NCT; ++ct, ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = (16 * it + lk + 4 * r) * kRcqMaxCols + 16 * ct + li;
            const double v = first ? w[u][r] : wsum[idx] + w[u][r];
            if (last)
              P[idx] = v;
            else
              wsum[idx] = v;
          }
#pragma unroll
      for (int c = 0; c < NZ; ++c)
        if (c < nx && lk == 0)
#pragma unroll
          for (int it = 0; it < NTI; ++it) {
            const int idx = (16 * it + li) * kRcqMaxCols + 16 * NTI + c;
            const double v = first ? z[it][c] : wsum[idx] + z[it][c];
            if (last)
              P[idx] = v;
            else
              wsum[idx] = v;
          }
    }
    if (wv < kGramWaves - 1) __syncthreads();
  }
}

// W = the sum of the nparts partials, element by element: wave q of a
// workgroup (16 waves) sums partials q, q + 16, ... of 64 consecutive
// elements in four interleaved running sums (added pairwise), and the 16
// waves' sums are added in wave order -- a fixed association.
constexpr int kRedW = 16;
__global__ __launch_bounds__(64 * kRedW) void k_rcq_reduce(int nparts,
                                                           const double *__restrict__ part,
                                                           double *__restrict__ W) {
  __shared__ double sh[kRedW][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int p = wave;
  for (; p + 3 * kRedW < nparts; p += 4 * kRedW)
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += part[(int64_t)(p + u * kRedW) * kPart + e];
  for (int u = 0; p < nparts; p += kRedW, ++u) s[u] += part[(int64_t)p * kPart + e];
  sh[wave][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (wave == 0) {
    double t = 0.0;
    for (int v = 0; v < kRedW; ++v) t += sh[v][lane];
    W[e] = t;
  }
}

// One wave: R1 = chol(G) (G = Q0^T Q0, the upper part of W), y = R1^{-T} z
// (z = Q0^T B, columns n .. n + nrhs of W), x = R^{-1} y with R = R1 R0.
// R0 and Rinv null: R0 = I (the normal equations: G = A^T A, z = A^T B,
// R = R1).
// Lane l holds column l of the working matrix in registers (g[i] = entry
// (i, l)); matrices of order n < 64 are padded to 64 with the identity, so
// every lane runs the same fully unrolled steps.
__global__ __launch_bounds__(64) void k_rcq_solve(int n, int nrhs, const double *__restrict__ W,
                                                  const double *__restrict__ R0, int ldr0,
                                                  const double *__restrict__ Rinv,
                                                  double *__restrict__ X, int64_t ldx,
                                                  double *__restrict__ Rout, int64_t ldr,
                                                  int *status) {
  constexpr int N = kRcqMaxN, L = kRcqMaxN + 1;
  __shared__ double r1[N * L];   // R1, row-major: r1[i L + l]
  __shared__ double rm[N * L];   // R0^{-1} staging, row-major: rm[i L + j]
  __shared__ double zs[kRcqMaxRhs * N];
  const int lane = threadIdx.x;
  double g[N];
#pragma unroll
  for (int i = 0; i < N; ++i)
    g[i] = lane < n ? (i <= lane ? W[i * kRcqMaxCols + lane] : 0.0) : (i == lane ? 1.0 : 0.0);
  for (int c = 0; c < nrhs; ++c) zs[c * N + lane] = lane < n ? W[lane * kRcqMaxCols + n + c] : 0.0;

  // right-looking Cholesky: at step j lane l forms R1[j][l] (l >= j), row j
  // goes to LDS, and every lane updates its column with it
  bool bad = false;
  double mydiag = 1.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double djj = read_lane(g[j], j);
    if (j < n && (!(djj > 0.0) || !isfinite(djj))) {
      bad = true;
      break;
    }
    const double rjj = sqrt(djj);
    const double rl = lane > j ? g[j] / rjj : (lane == j ? rjj : 0.0);
    g[j] = rl;
    if (lane == j) mydiag = rjj;
    r1[j * L + lane] = rl;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int i = j + 1; i < N; ++i) g[i] -= r1[j * L + i] * rl;
  }
  if (bad) {
    for (int c = 0; c < nrhs; ++c)
      if (lane < n) X[lane + (int64_t)c * ldx] = __longlong_as_double(0x7ff8000000000000LL);
    if (lane == 0) record_status(status, MS_ERR_SINGULAR);
    return;
  }
  // R1^T y = z, column oriented: y_i = z_i / R1[i][i], then lanes t > i
  // subtract R1[i][t] y_i (lane t's g[i])
  for (int c = 0; c < nrhs; ++c) {
    double y = zs[c * N + lane];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double yi = read_lane(y, i) / read_lane(mydiag, i);
      y = lane == i ? yi : (lane > i ? y - g[i] * yi : y);
    }
    zs[c * N + lane] = y;
  }
  // x = R^{-1} y with R = R1 R0, taken as R0^{-1} (R1^{-1} y): first the
  // back substitution with R1 (lanes t < i subtract R1[t][i] w_i), then the
  // product with R0^{-1} (Rinv, from the triangular inverse); without R0
  // (the normal equations) x = R1^{-1} y.  The straight-line product
  // R = R1 R0 is formed only when the caller asks for R.
  for (int c = 0; c < nrhs; ++c) {
    double y = zs[c * N + lane];
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      const double xi = read_lane(y, i) / read_lane(mydiag, i);
      y = lane == i ? xi : (lane < i ? y - r1[lane * L + i] * xi : y);
    }
    zs[c * N + lane] = y;
  }
  if (Rout && lane < n) {
    // R[i][lane] = sum_{q = i .. lane} R1[i][q] R0[q][lane] (rolled, from LDS
    // and R0 itself: an array indexed at run time must not share the
    // factorisation's registers, or all of them would live in scratch memory)
    for (int i = 0; i < n; ++i) {
      double acc = 0.0;
      if (R0)
        for (int q = i; q <= lane; ++q) acc += r1[i * L + q] * R0[q + (int64_t)lane * ldr0];
      else
        acc = i <= lane ? r1[i * L + lane] : 0.0;
      Rout[i + (int64_t)lane * ldr] = i <= lane ? acc : 0.0;
    }
  }
  __syncthreads();
  if (Rinv) {
    // R0^{-1} staged row-major (lane = column), then x_t = sum_q Rinv[t][q] w_q
    for (int i = 0; i < N; ++i) rm[i * L + lane] = Rinv[i * N + lane];
    __syncthreads();
    for (int c = 0; c < nrhs; ++c) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < N; ++q) acc[q & 3] += rm[lane * L + q] * zs[c * N + q];
      if (lane < n) X[lane + (int64_t)c * ldx] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  } else {
    for (int c = 0; c < nrhs; ++c)
      if (lane < n) X[lane + (int64_t)c * ldx] = zs[c * N + lane];
  }
}

}  // namespace

size_t rcq_partial_bytes(int grid) { return (size_t)grid * kPart * sizeof(double); }
int rcq_grid() { return dev_info().cus; }

hipError_t launch_rcq_trinv(int n, const double *R0, int ldr0, double *Rinv, int *status,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_rcq_trinv, dim3(1), dim3(256), 0, st, n, R0, ldr0, Rinv, status);
  return hipGetLastError();
}

template <typename TA>
hipError_t launch_rcq_gram(int64_t d, int n, int nrhs, const TA *A, int64_t lda, const TA *B,
                           int64_t ldb, const double *Rinv, double *part, int grid,
                           hipStream_t st) {
  if (n < 1 || n > kRcqMaxN || nrhs < 0 || n + nrhs > kRcqMaxCols) return hipErrorInvalidValue;
  const int nti = (n + 15) / 16, nx = n + nrhs - 16 * nti;
  const int extra = nx <= 0 ? 0 : (nx == 1 ? 2 : 1);
  if (nx > 16) return hipErrorInvalidValue;
#define MS_RCQ_CASE(T_, E_)                                                                 \
  case 3 * T_ + E_:                                                                         \
    if (Rinv)                                                                               \
      hipLaunchKernelGGL((k_rcq_gram<TA, T_, E_, false>), dim3(grid), dim3(64 * kGramWaves), \
                         0, st, d, n, nrhs, A, lda, B, ldb, Rinv, part);                    \
    else                                                                                    \
      hipLaunchKernelGGL((k_rcq_gram<TA, T_, E_, true>), dim3(grid), dim3(64 * kGramWaves),  \
                         0, st, d, n, nrhs, A, lda, B, ldb, Rinv, part);                    \
    break;
  switch (3 * nti + extra) {
    MS_RCQ_CASE(1, 0)
    MS_RCQ_CASE(1, 1)
    MS_RCQ_CASE(1, 2)
    MS_RCQ_CASE(2, 0)
    MS_RCQ_CASE(2, 1)
    MS_RCQ_CASE(2, 2)
    MS_RCQ_CASE(3, 0)
    MS_RCQ_CASE(3, 1)
    MS_RCQ_CASE(3, 2)
    MS_RCQ_CASE(4, 0)
    MS_RCQ_CASE(4, 1)
    MS_RCQ_CASE(4, 2)
  }
#undef MS_RCQ_CASE
  return hipGetLastError();
}
template hipError_t launch_rcq_gram<double>(int64_t, int, int, const double *, int64_t,
                                            const double *, int64_t, const double *, double *,
                                            int, hipStream_t);
template hipError_t launch_rcq_gram<float>(int64_t, int, int, const float *, int64_t,
                                           const float *, int64_t, const double *, double *, int,
                                           hipStream_t);

hipError_t launch_rcq_finish(int n, int nrhs, int nparts, const double *part, double *W,
                             const double *R0, int ldr0, const double *Rinv, double *X,
                             int64_t ldx, double *R, int64_t ldr, int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_rcq_reduce, dim3(kPart / 64), dim3(64 * kRedW), 0, st, nparts, part, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rcq_solve, dim3(1), dim3(64), 0, st, n, nrhs, W, R0, ldr0, Rinv, X, ldx,
                     R, ldr, status);
  return hipGetLastError();
}

}  // namespace ms
