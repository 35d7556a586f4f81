// rcq_wide.hip -- rand_cholQR least squares (Alg. 5) for wide problems
// (64 < n <= 256): the steps of randcholqr.hip with the multisketch's R0 of
// order up to 256.
//
//   R0^{-1}        one wave per column, back substitution against R0 (the
//                  QR factors' upper part);
//   Q0 = A R0^{-1} FP64 matrix cores, 64 x 64 output tiles (four waves of
//                  16 rows), the zero blocks of the triangular factor
//                  skipped, each tile transposed through LDS so that Q0's
//                  columns are written with full-line stores;
//   then Q0^T [Q0 | B], R1 = chol(Q0^T Q0), R1^T y = Q0^T B, x = R1^{-1} y,
//   x = R0^{-1} x by the wide normal-equation kernels (ne_wide.hip) on
//   V = [Q0 | B].
// Q0 is stored (d x n FP64 in the workspace): its Gram product reads it
// once more, instead of recomputing it in every tile task of that pass.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// Rinv (n x n, column-major, ld n; zero below the diagonal) = R0^{-1}, R0 the
// upper part of fact (ld ldf).  One wave per column j solves R0 x = e_j by
// column-oriented back substitution: x_l /= r_ll, then x_i -= r_il x_l for
// i < l, lane q holding x_q, x_{q+64}, x_{q+128}, x_{q+192}; the column r_.l
// is read with coalesced loads.  A zero or non-finite diagonal entry:
// MS_ERR_SINGULAR and a zero column.
__global__ __launch_bounds__(256) void k_trinv_wide(int n, const double *__restrict__ fact,
                                                    int64_t ldf, double *__restrict__ Rinv,
                                                    int *status) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (j >= n) return;
  double x[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = (lane + 64 * q == j) ? 1.0 : 0.0;
  bool sing = false;
  for (int l = j; l >= 0; --l) {
    const double dl = fact[l + (int64_t)l * ldf];
    if (!(dl != 0.0) || !isfinite(dl)) {
      sing = true;
      break;
    }
    const int ql = l >> 6, ll = l & 63;
    double v = x[0];
#pragma unroll
    for (int q = 1; q < 4; ++q)
      if (ql == q) v = x[q];
    const double xl = __shfl(v, ll, 64) / dl;
    const double *col = fact + (int64_t)l * ldf;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (i == l) x[q] = xl;
      else if (i < l) x[q] -= col[i] * xl;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    if (i < n) Rinv[i + (int64_t)j * n] = (!sing && i <= j) ? x[q] : 0.0;
  }
  if (sing && lane == 0) record_status(status, MS_ERR_SINGULAR);
}

// Q0 tile (64 rows from r0, 64 columns from c0) = A[r0:r0+64, 0:kend] Rinv[0:kend, c0:c0+64]
// with kend = min(n, c0 + 64) (the triangular factor's lower blocks are zero).
// Wave w takes rows r0 + 16 w .. + 15 and all four 16-column blocks.
template <typename TA>
__global__ __launch_bounds__(256) void k_q0_wide(int64_t d, int n, const TA *__restrict__ A,
                                                 int64_t lda, const double *__restrict__ Rinv,
                                                 double *__restrict__ Q0, int64_t ldq) {
  __shared__ double tile[64][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int kend = min(n, c0 + 64);
  const int64_t row = r0 + 16 * w + li;
  const bool rin = row < d;
  v4d acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kend; k0 += 4) {
    const int kk = k0 + lk;
    const double a = (rin && kk < kend) ? (double)gload(A + row + (int64_t)kk * lda) : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + 16 * j + li;
      const double b = (kk < kend && c < n) ? gload(Rinv + kk + (int64_t)c * n) : 0.0;
      acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
    }
  }
  // result register r of lane l: row (l / 16) + 4 r of the wave's 16, column l % 16
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) tile[16 * j + li][16 * w + lk + 4 * r] = acc[j][r];
  __syncthreads();
  // column c of the tile: 64 consecutive rows of Q0
  for (int t = threadIdx.x; t < 64 * 64; t += 256) {
    const int c = t >> 6, rr = t & 63;
    if (c0 + c < n && r0 + rr < d) Q0[(r0 + rr) + (int64_t)(c0 + c) * ldq] = tile[c][rr];
  }
}

}  // namespace

hipError_t launch_rcq_wide_q0(int64_t d, int n, ms_dtype a_dtype, const void *A, int64_t lda,
                              const double *fact, int64_t ldf, double *Rinv, double *Q0,
                              int *status, hipStream_t st) {
  if (n < 1 || n > kWideMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trinv_wide, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, fact, ldf,
                     Rinv, status);
  const dim3 grid((unsigned)((d + 63) / 64), (unsigned)((n + 63) / 64));
  if (a_dtype == MS_F64)
    hipLaunchKernelGGL(k_q0_wide<double>, grid, dim3(256), 0, st, d, n,
                       static_cast<const double *>(A), lda, (const double *)Rinv, Q0, d);
  else
    hipLaunchKernelGGL(k_q0_wide<float>, grid, dim3(256), 0, st, d, n,
                       static_cast<const float *>(A), lda, (const double *)Rinv, Q0, d);
  return hipGetLastError();
}

}  // namespace ms
