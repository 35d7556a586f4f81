// randcholqr.hip -- rand_cholQR least squares (Alg. 5, Sec. 6.3) after the
// multisketch: given R0 (the R factor of the sketched A, from the register
// QR), form Q0 = A R0^{-1}, the Gram matrix Q0^T Q0 and Q0^T B in one pass
// over A and B, then R1 = chol(Q0^T Q0), R = R1 R0, y = R1^{-T} Q0^T B and
// x = R^{-1} y.  The result is the least-squares optimum of min ||B - A x||:
// the sketch only preconditions.
//
// The pass over A is the dominant cost (2 d n^2 flops for Q0 and about as
// much for the Gram matrix, FP64): each persistent workgroup (4 waves) takes
// blocks of 64 rows; wave w forms the 16-row tile of Q0 = A R0^{-1} on the
// f64 matrix cores (R0^{-1} staged in LDS, its zero lower blocks skipped),
// the block [Q0 | B] goes to LDS, and the upper tiles of Q0^T [Q0 | B] are
// accumulated in registers across all the workgroup's blocks.  Q0 never
// reaches HBM: A and B are read once.  The workgroups' partial products are
// summed in a fixed order, then one workgroup factors and solves.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kLdr = 68;   // LDS row stride of R0^{-1} (doubles)
constexpr int kLdq = 84;   // LDS row stride of a [Q0 | B] block (doubles)
constexpr int kRows = 64;  // rows of A per block
constexpr int kPart = kRcqMaxN * kRcqMaxCols;  // doubles of one partial (64 x 80, row-major)

__device__ __forceinline__ v4d mma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// R0^{-1} (64 x 64, column-major, zero below the diagonal and outside n x n)
// by back substitution, one thread per column: R0 Rinv = I.
__global__ __launch_bounds__(64) void k_rcq_trinv(int n, const double *__restrict__ R0, int ldr0,
                                                  double *__restrict__ Rinv, int *status) {
  __shared__ double r0[kRcqMaxN * (kRcqMaxN + 1)];
  __shared__ double ri[kRcqMaxN * (kRcqMaxN + 1)];
  constexpr int L = kRcqMaxN + 1;
  for (int t = threadIdx.x; t < kRcqMaxN * kRcqMaxN; t += blockDim.x) {
    const int i = t % kRcqMaxN, j = t / kRcqMaxN;
    r0[i + j * L] = (i < n && j < n && i <= j) ? R0[i + (int64_t)j * ldr0] : 0.0;
    ri[i + j * L] = 0.0;
  }
  __syncthreads();
  const int j = threadIdx.x;
  bool bad = false;
  if (j < n) {
    const double djj = r0[j + j * L];
    bad = !(djj != 0.0) || !isfinite(djj);
    ri[j + j * L] = 1.0 / djj;
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int l = i + 1; l <= j; ++l) acc += r0[i + l * L] * ri[l + j * L];
      ri[i + j * L] = -acc / r0[i + i * L];
    }
  }
  if (bad) record_status(status, MS_ERR_SINGULAR);
  __syncthreads();
  for (int t = threadIdx.x; t < kRcqMaxN * kRcqMaxN; t += blockDim.x) {
    const int i = t % kRcqMaxN, jj = t / kRcqMaxN;
    Rinv[t] = ri[i + jj * L];
  }
}

// The fused pass.  NTI = column tiles of Q0 (n <= 16 NTI).  Partial of the
// workgroup: part[blockIdx.x] (64 x 80, row-major) holds the upper tiles of
// Q0^T [Q0 | B] over its blocks (tile (it, ct) for it <= ct; the lower
// off-diagonal tiles are not written).
template <typename TA, int NTI>
__global__ __launch_bounds__(256) void k_rcq_gram(int64_t d, int n, int nrhs,
                                                  const TA *__restrict__ A, int64_t lda,
                                                  const TA *__restrict__ B, int64_t ldb,
                                                  const double *__restrict__ Rinv,
                                                  double *__restrict__ part) {
  __shared__ double rinv[kRcqMaxN * kLdr];
  __shared__ double qb[kRows * kLdq];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int nc = n + nrhs;
  const int nct = (nc + 15) / 16;
  for (int t = tid; t < kRcqMaxN * kRcqMaxN; t += 256) {
    const int kk = t % kRcqMaxN, j = t / kRcqMaxN;
    rinv[kk * kLdr + j] = Rinv[t];
  }
  for (int t = tid; t < kRows * kLdq; t += 256) qb[t] = 0.0;
  __syncthreads();

  // this wave's tiles of Q0^T [Q0 | B]: (it, ct), it < NTI, it <= ct < nct,
  // numbered it-major; tile u goes to wave u % 4
  constexpr int kMaxTiles = 4;  // ceil(15 / 4): NTI <= 4 and nct <= 5
  int tit[kMaxTiles], tct[kMaxTiles];
  int ntile = 0;
  {
    int u = 0;
    for (int it = 0; it < NTI; ++it)
      for (int ct = it; ct < nct; ++ct, ++u)
        if (u % 4 == wave && ntile < kMaxTiles) {
          tit[ntile] = it;
          tct[ntile] = ct;
          ++ntile;
        }
  }
  v4d w[kMaxTiles];
#pragma unroll
  for (int u = 0; u < kMaxTiles; ++u) w[u] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t nblk = (d + kRows - 1) / kRows;
  // A fragments of a block for this wave: rows 16 wave + li, k = 4 ks + lk
  auto load_a = [&](int64_t blk, double(&fa)[4 * NTI]) {
    const int64_t row = blk * kRows + 16 * wave + li;
#pragma unroll
    for (int ks = 0; ks < 4 * NTI; ++ks) {
      const int kk = 4 * ks + lk;
      fa[ks] = (row < d && kk < n) ? (double)gload(A + row + (int64_t)kk * lda) : 0.0;
    }
  };
  double a[4 * NTI];
  int64_t blk = blockIdx.x;
  if (blk < nblk) load_a(blk, a);
  for (; blk < nblk; blk += gridDim.x) {
    const int64_t nb = blk + gridDim.x;
    double an[4 * NTI];
    if (nb < nblk) load_a(nb, an);
    // Q0 tile of this wave: rows 16 wave .. + 15, all columns; R0^{-1} is
    // upper triangular, so column tile jt needs k < 16 (jt + 1) only
#pragma unroll
    for (int jt = 0; jt < NTI; ++jt) {
      v4d q = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4 * (jt + 1); ++ks)
        q = mma64(a[ks], rinv[(4 * ks + lk) * kLdr + 16 * jt + li], q);
      const int col = 16 * jt + li;
      if (col < n)
#pragma unroll
        for (int r = 0; r < 4; ++r) qb[(16 * wave + lk + 4 * r) * kLdq + col] = q[r];
    }
    for (int t = tid; t < kRows * nrhs; t += 256) {
      const int row = t % kRows, c = t / kRows;
      const int64_t grow = blk * kRows + row;
      qb[row * kLdq + n + c] = grow < d ? (double)gload(B + grow + (int64_t)c * ldb) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxTiles; ++u)
      if (u < ntile) {
        const int ci = 16 * tit[u] + li, cc = 16 * tct[u] + li;
#pragma unroll
        for (int ks = 0; ks < kRows / 4; ++ks) {
          const int row = 4 * ks + lk;
          w[u] = mma64(qb[row * kLdq + ci], qb[row * kLdq + cc], w[u]);
        }
      }
    __syncthreads();
    if (nb < nblk)
#pragma unroll
      for (int ks = 0; ks < 4 * NTI; ++ks) a[ks] = an[ks];
  }
  double *P = part + (int64_t)blockIdx.x * kPart;
#pragma unroll
  for (int u = 0; u < kMaxTiles; ++u)
    if (u < ntile)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        P[(16 * tit[u] + lk + 4 * r) * kRcqMaxCols + 16 * tct[u] + li] = w[u][r];
}

// W = the sum of the nparts partials, element by element: wave q of a
// workgroup sums partials q, q + 4, ... of 64 consecutive elements, and the
// four sums are added in wave order (a fixed association).
__global__ __launch_bounds__(256) void k_rcq_reduce(int nparts, const double *__restrict__ part,
                                                    double *__restrict__ W) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  double s = 0.0;
  for (int p = wave; p < nparts; p += 4) s += part[(int64_t)p * kPart + e];
  sh[wave][lane] = s;
  __syncthreads();
  if (wave == 0) W[e] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

// One workgroup: R1 = chol(G) (G = Q0^T Q0, upper part of W), R = R1 R0,
// y = R1^{-T} z (z = Q0^T B, columns n .. n + nrhs of W), x = R^{-1} y.
__global__ __launch_bounds__(256) void k_rcq_solve(int n, int nrhs, const double *__restrict__ W,
                                                   const double *__restrict__ R0, int ldr0,
                                                   double *__restrict__ X, int64_t ldx,
                                                   double *__restrict__ Rout, int64_t ldr,
                                                   int *status) {
  constexpr int L = kRcqMaxN + 1;
  __shared__ double g[kRcqMaxN * L];   // g[i + j L]: R1 in the upper triangle
  __shared__ double r0[kRcqMaxN * L];
  __shared__ double rr[kRcqMaxN * L];  // R = R1 R0
  __shared__ double z[kRcqMaxN * 16];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int t = tid; t < n * n; t += blockDim.x) {
    const int i = t % n, j = t / n;
    // the upper triangle of Q0^T Q0 (row i, column j of the row-major W)
    g[i + j * L] = i <= j ? W[i * kRcqMaxCols + j] : 0.0;
    r0[i + j * L] = i <= j ? R0[i + (int64_t)j * ldr0] : 0.0;
  }
  for (int t = tid; t < n * nrhs; t += blockDim.x) {
    const int i = t % n, c = t / n;
    z[i + c * kRcqMaxN] = W[i * kRcqMaxCols + n + c];
  }
  __syncthreads();
  // right-looking Cholesky, one barrier per column: step j updates the
  // trailing rows with the undivided row j, and row j is scaled at step j + 1
  for (int j = 0; j < n; ++j) {
    const double djj = g[j + j * L];
    if (!(djj > 0.0) || !isfinite(djj)) {
      if (tid == 0) bad = 1;
      break;
    }
    const double inv = 1.0 / djj;
    const int m = n - 1 - j;  // trailing order
    for (int t = tid; t < m * m; t += blockDim.x) {
      const int i = j + 1 + t % m, c = j + 1 + t / m;
      if (i <= c) g[i + c * L] -= g[j + i * L] * g[j + c * L] * inv;
    }
    __syncthreads();
    const double rjj = sqrt(djj);
    for (int c = j + tid; c < n; c += blockDim.x) g[j + c * L] = c == j ? rjj : g[j + c * L] / rjj;
    __syncthreads();
  }
  if (bad) {
    for (int t = tid; t < n * nrhs; t += blockDim.x)
      X[t % n + (int64_t)(t / n) * ldx] = __longlong_as_double(0x7ff8000000000000LL);
    if (tid == 0) record_status(status, MS_ERR_SINGULAR);
    return;
  }
  // R = R1 R0
  for (int t = tid; t < n * n; t += blockDim.x) {
    const int i = t % n, j = t / n;
    double acc = 0.0;
    if (i <= j)
      for (int q = i; q <= j; ++q) acc += g[i + q * L] * r0[q + j * L];
    rr[i + j * L] = acc;
    if (Rout) Rout[i + (int64_t)j * ldr] = acc;
  }
  __syncthreads();
  // per right-hand side, one wave: R1^T y = z (forward), then R x = y
  const int lane = tid & 63, wave = tid >> 6;
  for (int c = wave; c < nrhs; c += 4) {
    double *y = z + c * kRcqMaxN;
    for (int i = 0; i < n; ++i) {
      const double yi = y[i] / g[i + i * L];
      if (lane == 0) y[i] = yi;
      for (int t = i + 1 + lane; t < n; t += 64) y[t] -= g[i + t * L] * yi;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    for (int i = n - 1; i >= 0; --i) {
      const double xi = y[i] / rr[i + i * L];
      if (lane == 0) {
        y[i] = xi;
        X[i + (int64_t)c * ldx] = xi;
      }
      for (int t = lane; t < i; t += 64) y[t] -= rr[t + i * L] * xi;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  }
}

}  // namespace

size_t rcq_partial_bytes(int grid) { return (size_t)grid * kPart * sizeof(double); }
int rcq_grid() { return dev_info().cus; }

hipError_t launch_rcq_trinv(int n, const double *R0, int ldr0, double *Rinv, int *status,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_rcq_trinv, dim3(1), dim3(64), 0, st, n, R0, ldr0, Rinv, status);
  return hipGetLastError();
}

template <typename TA>
hipError_t launch_rcq_gram(int64_t d, int n, int nrhs, const TA *A, int64_t lda, const TA *B,
                           int64_t ldb, const double *Rinv, double *part, int grid,
                           hipStream_t st) {
  if (n < 1 || n > kRcqMaxN || nrhs < 0 || n + nrhs > kRcqMaxCols) return hipErrorInvalidValue;
  const int nti = (n + 15) / 16;
#define MS_RCQ_CASE(T_)                                                                      \
  case T_:                                                                                   \
    hipLaunchKernelGGL((k_rcq_gram<TA, T_>), dim3(grid), dim3(256), 0, st, d, n, nrhs, A, lda, \
                       B, ldb, Rinv, part);                                                  \
    break;
  switch (nti) {
    MS_RCQ_CASE(1)
    MS_RCQ_CASE(2)
    MS_RCQ_CASE(3)
    MS_RCQ_CASE(4)
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
                             const double *R0, int ldr0, double *X, int64_t ldx, double *R,
                             int64_t ldr, int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_rcq_reduce, dim3(kPart / 64), dim3(256), 0, st, nparts, part, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rcq_solve, dim3(1), dim3(256), 0, st, n, nrhs, W, R0, ldr0, X, ldx, R,
                     ldr, status);
  return hipGetLastError();
}

}  // namespace ms
