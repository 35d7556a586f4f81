// qr.hip -- FP64 Householder QR least squares of the small sketched system
// (Alg. 1 steps 2-3 of Higgins, Boman, Yamazaki, arXiv 2508.14209; the paper
// runs GeQRF + OrMQR + a triangular solve, Sec. 6.1 and 6.3).
//
// One workgroup of 16 waves owns the whole m x (n + nrhs) system [W | Bm]:
// reflector j is formed by wave 0 (norm by a wave reduction, LAPACK geqr2
// convention: beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta,
// v = x/(alpha - beta) with v_0 = 1), then every wave applies it to its own
// columns (one column per wave at a time: a dot product by wave reduction and
// an axpy), so the right-hand sides receive Q^T as the factorisation runs.
// Back substitution is one wave per right-hand side.  The system lives in LDS
// when it fits and in the workspace otherwise.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Back substitution R x = y for one right-hand side y (length >= n, in
// memory), by one wave; x written to X (stride 1).  y is overwritten.
__device__ __forceinline__ void wave_back_substitute(int n, const double *R, int64_t ldr,
                                                     double *y, double *X) {
  const int lane = threadIdx.x & 63;
  for (int i = n - 1; i >= 0; --i) {
    const double xi = y[i] / R[i + (int64_t)i * ldr];
    for (int t = lane; t < i; t += 64) y[t] -= R[t + (int64_t)i * ldr] * xi;
    if (lane == 0) X[i] = xi;
    __threadfence_block();
  }
}

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void k_qr_solve(int m, int n, int nrhs, const double *__restrict__ W,
                                                   int64_t ldw, const double *__restrict__ Bm,
                                                   int64_t ldb, double *__restrict__ X, int64_t ldx,
                                                   double *__restrict__ R, int64_t ldr,
                                                   double *__restrict__ tau_out,
                                                   double *__restrict__ fact_out, double *gmat,
                                                   int *status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *Mx = IN_LDS ? reinterpret_cast<double *>(smem_raw) : gmat;
  __shared__ double s_tau;
  __shared__ int s_singular;
  const int nc = n + nrhs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  for (int64_t t = tid; t < (int64_t)m * nc; t += blockDim.x) {
    const int c = (int)(t / m);
    const int i = (int)(t - (int64_t)c * m);
    Mx[t] = c < n ? W[i + (int64_t)c * ldw] : Bm[i + (int64_t)(c - n) * ldb];
  }
  if (tid == 0) s_singular = 0;
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    double *vj = Mx + (int64_t)j * m;
    if (wave == 0) {
      double part = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) part += vj[i] * vj[i];
      const double xn2 = wave_sum(part);
      const double alpha = vj[j];
      double tau = 0.0;
      if (xn2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + xn2);
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int i = j + 1 + lane; i < m; i += 64) vj[i] *= scal;
        if (lane == 0) vj[j] = beta;
      }
      if (lane == 0) {
        s_tau = tau;
        if (tau_out) tau_out[j] = tau;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < nc; c += nw) {
        double *cc = Mx + (int64_t)c * m;
        double part = lane == 0 ? cc[j] : 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) part += vj[i] * cc[i];
        const double w = wave_sum(part) * tau;
        if (lane == 0) cc[j] -= w;
        for (int i = j + 1 + lane; i < m; i += 64) cc[i] -= w * vj[i];
      }
    }
    __syncthreads();
  }

  // factors for later solves with new right-hand sides
  if (fact_out)
    for (int64_t t = tid; t < (int64_t)m * n; t += blockDim.x) fact_out[t] = Mx[t];
  if (R)
    for (int64_t t = tid; t < (int64_t)n * n; t += blockDim.x) {
      const int c = (int)(t / n), i = (int)(t - (int64_t)c * n);
      R[i + (int64_t)c * ldr] = i <= c ? Mx[i + (int64_t)c * m] : 0.0;
    }
  for (int i = tid; i < n; i += blockDim.x) {
    const double r = Mx[i + (int64_t)i * m];
    if (r == 0.0 || !isfinite(r)) s_singular = 1;
  }
  __syncthreads();
  if (s_singular) {
    for (int64_t t = tid; t < (int64_t)n * nrhs; t += blockDim.x) {
      const int c = (int)(t / n), i = (int)(t - (int64_t)c * n);
      X[i + (int64_t)c * ldx] = __longlong_as_double(0x7ff8000000000000LL);
    }
    if (tid == 0) record_status(status, MS_ERR_SINGULAR);
    return;
  }
  for (int c = wave; c < nrhs; c += nw)
    wave_back_substitute(n, Mx, m, Mx + (int64_t)(n + c) * m, X + (int64_t)c * ldx);
}

size_t qr_workspace_bytes(int64_t m, int64_t n, int64_t nrhs) {
  return (size_t)m * (size_t)(n + nrhs) * sizeof(double);
}

hipError_t launch_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W, int64_t ldw,
                           const double *Bm, int64_t ldb, double *X, int64_t ldx, double *R,
                           int64_t ldr, double *tau_out, double *fact_out, void *qr_ws,
                           int *status, hipStream_t st) {
  const DevInfo &di = dev_info();
  const size_t bytes = qr_workspace_bytes(m, n, nrhs);
  if (bytes + 1024 <= (size_t)di.lds_per_block) {
    hipError_t e = allow_dynamic_lds((const void *)k_qr_solve<true>, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_qr_solve<true>, dim3(1), dim3(1024), bytes, st, (int)m, (int)n,
                       (int)nrhs, W, ldw, Bm, ldb, X, ldx, R, ldr, tau_out, fact_out,
                       (double *)nullptr, status);
  } else {
    hipLaunchKernelGGL(k_qr_solve<false>, dim3(1), dim3(1024), 0, st, (int)m, (int)n, (int)nrhs,
                       W, ldw, Bm, ldb, X, ldx, R, ldr, tau_out, fact_out, (double *)qr_ws,
                       status);
  }
  return hipGetLastError();
}

// Apply H_0 ... H_{n-1} (stored in fact/tau) to each right-hand side, one
// wave per column, then back-substitute with R from fact.
__global__ __launch_bounds__(1024) void k_qr_apply_solve(int m, int n, int nrhs,
                                                         const double *__restrict__ fact,
                                                         const double *__restrict__ tau,
                                                         double *Bm, double *__restrict__ X,
                                                         int64_t ldx, int *status) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __shared__ int s_singular;
  if (threadIdx.x == 0) s_singular = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = fact[i + (int64_t)i * m];
    if (r == 0.0 || !isfinite(r)) s_singular = 1;
  }
  __syncthreads();
  if (s_singular) {
    for (int64_t t = threadIdx.x; t < (int64_t)n * nrhs; t += blockDim.x) {
      const int c = (int)(t / n), i = (int)(t - (int64_t)c * n);
      X[i + (int64_t)c * ldx] = __longlong_as_double(0x7ff8000000000000LL);
    }
    if (threadIdx.x == 0) record_status(status, MS_ERR_SINGULAR);
    return;
  }
  for (int c = wave; c < nrhs; c += nw) {
    double *b = Bm + (int64_t)c * m;
    for (int j = 0; j < n; ++j) {
      const double tj = tau[j];
      if (tj == 0.0) continue;
      const double *v = fact + (int64_t)j * m;
      double part = lane == 0 ? b[j] : 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) part += v[i] * b[i];
      const double w = wave_sum(part) * tj;
      if (lane == 0) b[j] -= w;
      for (int i = j + 1 + lane; i < m; i += 64) b[i] -= w * v[i];
      __threadfence_block();
    }
    wave_back_substitute(n, fact, m, b, X + (int64_t)c * ldx);
  }
}

hipError_t launch_qr_apply_solve(int64_t m, int64_t n, int64_t nrhs, const double *fact,
                                 const double *tau, double *Bm, double *X, int64_t ldx,
                                 int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_qr_apply_solve, dim3(1), dim3(1024), 0, st, (int)m, (int)n, (int)nrhs,
                     fact, tau, Bm, X, ldx, status);
  return hipGetLastError();
}

}  // namespace ms
