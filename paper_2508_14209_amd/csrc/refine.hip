// refine.hip -- FP64 residual of the mixed-precision least-squares path.
//
// r = B - A X in FP64: A (d x n, FP32 or FP64, column-major) is promoted
// exactly, X (n x nrhs) is FP64, B has A's type, every product and sum is
// FP64.  Each thread takes four consecutive rows with one 16-byte load per
// column of A (a wave reads 1 KB of a column at a time) and keeps the 4 x
// nrhs sums in registers; X is staged in LDS.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

// Four consecutive rows of a column, promoted to FP64.  The vector loads are
// aligned to the element only (a dword-aligned multi-dword global load is
// legal on CDNA), so a column may start at any element.
template <typename TA>
struct Rows4 {
  static __device__ __forceinline__ void load(const TA *p, double v[4]) {
    typedef TA V __attribute__((ext_vector_type(4), aligned(sizeof(TA))));
    const V a = gload(reinterpret_cast<const V *>(p));
    v[0] = (double)a.x;
    v[1] = (double)a.y;
    v[2] = (double)a.z;
    v[3] = (double)a.w;
  }
};
template <>
struct Rows4<double> {
  static __device__ __forceinline__ void load(const double *p, double v[4]) {
    typedef double V __attribute__((ext_vector_type(2), aligned(8)));
    const V a = gload(reinterpret_cast<const V *>(p));
    const V b = gload(reinterpret_cast<const V *>(p + 2));
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
  }
};

constexpr int kResXlds = 8192;  // doubles of X staged in LDS (64 KB)

template <typename TA, bool XLDS>
__global__ __launch_bounds__(256) void k_residual(int64_t d, int n, int nrhs,
                                                  const TA *__restrict__ A, int64_t lda,
                                                  const TA *__restrict__ B, int64_t ldb,
                                                  const double *__restrict__ X, int64_t ldx,
                                                  double *__restrict__ r, int64_t ldr) {
  constexpr int RH = 8;
  __shared__ double xs[XLDS ? kResXlds : 1];  // xs[j * RH + c] = X[j, c]
  if (XLDS) {
    for (int t = threadIdx.x; t < n * nrhs; t += blockDim.x) {
      const int c = t / n, j = t - c * n;
      xs[j * RH + c] = X[j + (int64_t)c * ldx];
    }
    __syncthreads();
  }
  auto xv = [&](int j, int c) { return XLDS ? xs[j * RH + c] : X[j + (int64_t)c * ldx]; };
  for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i0 < d;
       i0 += (int64_t)gridDim.x * blockDim.x * 4) {
    const bool vec = i0 + 4 <= d;
    const int rows = (int)min((int64_t)4, d - i0);
    double acc[4][RH];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < RH; ++c) acc[q][c] = 0.0;
    if (vec) {
      int j = 0;
      for (; j + 4 <= n; j += 4) {
        double a[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) Rows4<TA>::load(A + i0 + (int64_t)(j + u) * lda, a[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int c = 0; c < RH; ++c)
            if (c < nrhs) {
              const double x = xv(j + u, c);
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[q][c] += a[u][q] * x;
            }
      }
      for (; j < n; ++j) {
        double a[4];
        Rows4<TA>::load(A + i0 + (int64_t)j * lda, a);
#pragma unroll
        for (int c = 0; c < RH; ++c)
          if (c < nrhs) {
            const double x = xv(j, c);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q][c] += a[q] * x;
          }
      }
#pragma unroll
      for (int c = 0; c < RH; ++c)
        if (c < nrhs) {
          double b[4];
          Rows4<TA>::load(B + i0 + (int64_t)c * ldb, b);
#pragma unroll
          for (int q = 0; q < 4; ++q) r[i0 + q + (int64_t)c * ldr] = b[q] - acc[q][c];
        }
    } else {
      for (int j = 0; j < n; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q < rows) {
            const double a = (double)A[i0 + q + (int64_t)j * lda];
#pragma unroll
            for (int c = 0; c < RH; ++c)
              if (c < nrhs) acc[q][c] += a * xv(j, c);
          }
#pragma unroll
      for (int c = 0; c < RH; ++c)
        if (c < nrhs)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q < rows) r[i0 + q + (int64_t)c * ldr] = (double)B[i0 + q + (int64_t)c * ldb] - acc[q][c];
    }
  }
}

template <typename TA>
static hipError_t launch_residual_t(int64_t d, int64_t n, int64_t nrhs, const TA *A, int64_t lda,
                                    const TA *B, int64_t ldb, const double *X, int64_t ldx,
                                    double *r, int64_t ldr, hipStream_t st) {
  if (nrhs > 8) return hipErrorInvalidValue;
  if (d <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((d + 1023) / 1024, (int64_t)dev_info().cus * 8);
  if (n * 8 <= kResXlds)
    hipLaunchKernelGGL((k_residual<TA, true>), dim3(grid), dim3(256), 0, st, d, (int)n, (int)nrhs,
                       A, lda, B, ldb, X, ldx, r, ldr);
  else
    hipLaunchKernelGGL((k_residual<TA, false>), dim3(grid), dim3(256), 0, st, d, (int)n,
                       (int)nrhs, A, lda, B, ldb, X, ldx, r, ldr);
  return hipGetLastError();
}

hipError_t launch_residual_f32(int64_t d, int64_t n, int64_t nrhs, const float *A, int64_t lda,
                               const float *B, int64_t ldb, const double *X, int64_t ldx,
                               double *r, int64_t ldr, hipStream_t st) {
  return launch_residual_t<float>(d, n, nrhs, A, lda, B, ldb, X, ldx, r, ldr, st);
}

hipError_t launch_residual_f64(int64_t d, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                               const double *B, int64_t ldb, const double *X, int64_t ldx,
                               double *r, int64_t ldr, hipStream_t st) {
  return launch_residual_t<double>(d, n, nrhs, A, lda, B, ldb, X, ldx, r, ldr, st);
}

// Residuals of a batch: item = (problem, kBatchResRows rows) taken in
// sub-blocks of 1024 rows, four rows per thread (16-byte loads of A and B
// when aligned), X staged in LDS once per item; B has A's type.  r_p is
// d x nrhs, column-major, ld d.
template <typename TA>
__global__ __launch_bounds__(256) void k_batch_residual(
    int count, const ms_problem *__restrict__ P, const BatchEntry *__restrict__ E,
    const BatchTotals *__restrict__ tot, unsigned char *__restrict__ rarea) {
  constexpr int RH = kBatchMaxRefineRhs;
  __shared__ double xs[kBatchMaxCols * RH];  // xs[j * RH + c] = X[j, c]
  const int64_t total = tot->res_items;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = batch_find_m<&BatchEntry::res_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    if (!e.refine) continue;   // converged in an earlier step
    const int n = (int)Q.n, nrhs = (int)Q.nrhs;
    __syncthreads();  // the previous item's reads of xs are done
    for (int t = threadIdx.x; t < n * nrhs; t += blockDim.x) {
      const int c = t / n, j = t - c * n;
      xs[j * RH + c] = gload(Q.X + j + (int64_t)c * Q.ldx);
    }
    __syncthreads();
    for (int64_t sub = 0; sub < kBatchResRows; sub += 4 * (int64_t)blockDim.x) {
      const int64_t i0 = (it - e.res_start) * kBatchResRows + sub + (int64_t)threadIdx.x * 4;
      if (i0 >= Q.d) break;
      const TA *A = static_cast<const TA *>(Q.A);
      const TA *B = static_cast<const TA *>(Q.B);
      double *r = reinterpret_cast<double *>(rarea + e.r_off);
      const bool vec = i0 + 4 <= Q.d;
      const int rows = (int)min((int64_t)4, Q.d - i0);
      double acc[4][RH];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < RH; ++c) acc[q][c] = 0.0;
      if (vec) {
        int j = 0;
        for (; j + 4 <= n; j += 4) {
          double a[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u) Rows4<TA>::load(A + i0 + (int64_t)(j + u) * Q.lda, a[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < RH; ++c)
              if (c < nrhs) {
                const double x = xs[(j + u) * RH + c];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q][c] += a[u][q] * x;
              }
        }
        for (; j < n; ++j) {
          double a[4];
          Rows4<TA>::load(A + i0 + (int64_t)j * Q.lda, a);
#pragma unroll
          for (int c = 0; c < RH; ++c)
            if (c < nrhs) {
              const double x = xs[j * RH + c];
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[q][c] += a[q] * x;
            }
        }
#pragma unroll
        for (int c = 0; c < RH; ++c)
          if (c < nrhs) {
            double b[4];
            Rows4<TA>::load(B + i0 + (int64_t)c * Q.ldb, b);
#pragma unroll
            for (int q = 0; q < 4; ++q) r[i0 + q + (int64_t)c * Q.d] = b[q] - acc[q][c];
          }
      } else {
        for (int j = 0; j < n; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q < rows) {
              const double a = (double)gload(A + i0 + q + (int64_t)j * Q.lda);
#pragma unroll
              for (int c = 0; c < RH; ++c)
                if (c < nrhs) acc[q][c] += a * xs[j * RH + c];
            }
#pragma unroll
        for (int c = 0; c < RH; ++c)
          if (c < nrhs)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (q < rows)
                r[i0 + q + (int64_t)c * Q.d] = (double)gload(B + i0 + q + (int64_t)c * Q.ldb) - acc[q][c];
      }
    }
  }
}

template <typename TA>
hipError_t launch_batch_residual(int count, const ms_problem *P, const BatchEntry *E,
                                 const BatchTotals *tot, unsigned char *rarea, int grid,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_batch_residual<TA>, dim3(grid), dim3(256), 0, st, count, P, E, tot,
                     rarea);
  return hipGetLastError();
}
template hipError_t launch_batch_residual<float>(int, const ms_problem *, const BatchEntry *,
                                                 const BatchTotals *, unsigned char *, int,
                                                 hipStream_t);
template hipError_t launch_batch_residual<double>(int, const ms_problem *, const BatchEntry *,
                                                  const BatchTotals *, unsigned char *, int,
                                                  hipStream_t);

// X += dX (n x nrhs).
__global__ void k_axpy_update(int n, int nrhs, const double *__restrict__ dX, double *X,
                              int64_t ldx) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * nrhs) return;
  const int c = (int)(t / n), i = (int)(t - (int64_t)c * n);
  X[i + (int64_t)c * ldx] += dX[t];
}

hipError_t launch_axpy_update(int64_t n, int64_t nrhs, const double *dX, double *X, int64_t ldx,
                              hipStream_t st) {
  const int64_t t = n * nrhs;
  hipLaunchKernelGGL(k_axpy_update, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, (int)n,
                     (int)nrhs, dX, X, ldx);
  return hipGetLastError();
}

}  // namespace ms
