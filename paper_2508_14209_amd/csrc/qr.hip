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
#include <type_traits>
#include <utility>

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

// ------------------------------------------------------------------ register-resident QR
// Back substitution R x = y by one wave, y held in registers (lane l owns
// rows l + 64 r): per row a lane read, one division and one update per lane.
template <int RPL>
__device__ __forceinline__ void wave_back_substitute_reg(int n, const double *R, int ldr,
                                                         const double *ysrc, double *X) {
  const int lane = threadIdx.x & 63;
  double y[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int t = lane + 64 * r;
    y[r] = t < n ? ysrc[t] : 0.0;
  }
  for (int i = n - 1; i >= 0; --i) {
    double yl = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (r == (i >> 6)) yl = y[r];
    const double xi = read_lane(yl, i & 63) / R[i + i * ldr];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int t = lane + 64 * r;
      if (t < i) y[r] -= R[t + i * ldr] * xi;
    }
    if (lane == 0) X[i] = xi;
  }
}

// Sum over the 16 lanes of a DPP row (quad swaps, half-row and row mirrors);
// every lane of the row receives the same bits, since each step adds the same
// two partial sums in either order.
__device__ __forceinline__ double row_allsum(double v) {
  v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}
// The value of lane i ^ 16 (ds_swizzle in bit-mask mode: and 0x1f, xor 0x10).
__device__ __forceinline__ double swap_rows(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(u & 0xffffffffLL), 0x401f);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(u >> 32), 0x401f);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over a group of GW (16 or 32) lanes, the same bits in every lane of it.
template <int GW>
__device__ __forceinline__ double group_allsum(double v) {
  v = row_allsum(v);
  if (GW == 32) v += swap_rows(v);
  return v;
}

// Square root and reciprocal for the reflector's scalars: a single-precision
// hardware estimate (v_rsq_f32, v_rcp_f32, relative error near 2^-23; the
// double-precision estimates have a much longer latency on this chip)
// refined by Newton's method in double precision: for the reciprocal
// y <- y + y (1 - x y) twice; for the square root Goldschmidt's coupled
// iteration g -> sqrt(s), h -> 1 / (2 sqrt(s)) twice, then one residual
// correction g + h (s - g^2).  Each result is within an ulp or two of the
// correctly rounded one.  Outside [2^-120, 2^120] (beyond the single-precision
// range) the library operations are used; the argument is uniform across the
// wave, so that is a scalar branch.
__device__ __forceinline__ double qr_sqrt(double s) {
  if (!(s >= 0x1p-120 && s <= 0x1p120)) return sqrt(s);
  const double y = (double)__builtin_amdgcn_rsqf((float)s);
  double g = s * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, s);
  return fma(d, h, g);
}
__device__ __forceinline__ double qr_rcp(double x) {
  const double ax = fabs(x);
  if (!(ax >= 0x1p-120 && ax <= 0x1p120)) return 1.0 / x;
  double y = (double)__builtin_amdgcn_rcpf((float)x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// f(std::integral_constant<int, I>) for I = 0, ..., N - 1, unrolled.
template <typename F, int... I>
__device__ __forceinline__ void qr_static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void qr_static_for(F &&f) {
  qr_static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int ROWS>
struct QrShared {
  double vbuf[2][ROWS];
  double taubuf[2];
  int singular;
};

// Householder QR least squares (the factorisation of the sketched system,
// Section 2 and Algorithm 1's final solve) with [W | Bm] (m x nc, nc = n +
// nrhs) held in registers.  The NW waves form NG = 64 NW / GW groups of GW
// lanes (one or two DPP rows): group g owns columns g + NG s (s < S), and lane
// l of a group rows l + GW r (r < R).  A column's inner product with a
// reflector is R fused multiply-adds per lane (in up to four independent
// chains) and a sum over the group that DPP steps (and, for 32 lanes, one
// swizzle) give to every lane of it.  Reflector j is built by the group
// owning column j and published through a double-buffered LDS vector: one
// barrier per column.  Look-ahead: after the barrier that publishes
// reflector j, the wave owning column j + 1 applies reflector j to that
// column first, builds and publishes reflector j + 1, and only then updates
// its other columns, so the serial part of a step (norm, square root,
// division) overlaps the other waves' updates.  The input is either [W | Bm]
// or, when part (FP64) or part32 (FP32) is given, the sum in split order of
// nsplit split-K partial blocks of an m x nc product -- the same sum, in the
// same precision, as the separate split reduction.  R and the transformed
// right-hand sides go to LDS (rs: dynamic LDS of n x nc doubles) for the back
// substitution; status2 (may be null) also receives a singular-R report.
template <int NW, int GW, int R, int S>
__device__ __forceinline__ void qr_reg_body(int m, int n, int nrhs, const double *__restrict__ W,
                                            int64_t ldw, const double *__restrict__ Bm,
                                            int64_t ldb, const double *__restrict__ part,
                                            const float *__restrict__ part32, int nsplit,
                                            double *__restrict__ X, int64_t ldx,
                                            double *__restrict__ Rout, int64_t ldr,
                                            double *__restrict__ tau_out,
                                            double *__restrict__ fact_out, int *status,
                                            int *status2, double *rs, QrShared<GW * R> &sh) {
  constexpr int NG = NW * 64 / GW;   // groups
  constexpr int GPW = 64 / GW;       // groups per wave
  // independent partial sums (two when the columns leave few registers)
  constexpr int NP = R >= 4 && S <= 3 ? 4 : (R >= 2 ? 2 : 1);
  auto &vbuf = sh.vbuf;
  auto &taubuf = sh.taubuf;
  int &s_singular = sh.singular;
  const int nc = n + nrhs;
  const int lane = threadIdx.x & 63;
  // uniform across a wave; saying so keeps the per-column conditions scalar
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int gl = lane % GW;
  const int grp = wave * GPW + lane / GW;
  const int64_t MN = (int64_t)m * nc;

  double a[S][R];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int c = grp + NG * s;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = gl + GW * r;
      double x = 0.0;
      if (i < m && c < nc) {
        const int64_t o = i + (int64_t)c * m;
        if (part) {
          x = part[o];
          for (int z = 1; z < nsplit; ++z) x = x + part[o + z * MN];
        } else if (part32) {
          float x32 = part32[o];
          for (int z = 1; z < nsplit; ++z) x32 = x32 + part32[o + z * MN];
          x = (double)x32;
        } else {
          x = c < n ? W[i + (int64_t)c * ldw] : Bm[i + (int64_t)(c - n) * ldb];
        }
      }
      a[s][r] = x;
    }
  }
  if (threadIdx.x == 0) s_singular = 0;

  auto owner_wave = [&](int j) { return (j % NG) / GPW; };
  // Reflector j from column j, slot col of the owning wave (every group of
  // the wave runs the steps on its own column; only the owner publishes and
  // keeps the result).  With t = |alpha| + ||x||: tau = t / ||x|| and the
  // scale of v below the diagonal is sign(alpha) / t, from one product with
  // the reciprocal of ||x|| t.  Lane gl holds rows gl + GW r: the blocks
  // r < j / GW lie wholly above row j and r > j / GW wholly below it, so when
  // the block RJ = j / GW is a compile-time constant only that block needs a
  // per-lane condition; RJ = -1 is the general form with a condition on every
  // row.
  auto build_rows = [&](auto rjc, int j, double(&col)[R]) {
    constexpr int RJ = decltype(rjc)::value;
    const int og = (j % NG) % GPW;
    const int olane = og * GW;
    const bool own = lane / GW == og;
    auto below = [&](int r) { return RJ >= 0 ? (r > RJ || (r == RJ && gl + GW * r > j)) : gl + GW * r > j; };
    auto diag = [&](int r) { return RJ >= 0 ? (r == RJ && gl + GW * r == j) : gl + GW * r == j; };
    double p[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) p[q] = 0.0;
    double av = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (RJ >= 0 && r < RJ) continue;
      if (below(r)) p[r % NP] += col[r] * col[r];
      if (RJ >= 0 ? r == RJ : r == j / GW) av = col[r];
    }
    double ps = p[0];
#pragma unroll
    for (int q = 1; q < NP; ++q) ps += p[q];
    const double xn2 = read_lane(group_allsum<GW>(ps), olane);
    const double alpha = read_lane(av, olane + j % GW);
    double tau = 0.0, beta = alpha, scal = 0.0;
    if (xn2 != 0.0) {
      const double nrm = qr_sqrt(alpha * alpha + xn2);
      const double tt = fabs(alpha) + nrm;
      const double qq = qr_rcp(nrm * tt);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = tt * tt * qq;
      scal = (alpha >= 0.0 ? nrm : -nrm) * qq;
    }
    const int buf = j & 1;
    // branch-free: with x = 0 (tau = 0, beta = alpha) the column keeps its
    // values (scale 1), and tau = 0 makes every update with v a no-op
    const double sv = xn2 != 0.0 ? scal : 1.0;
    if (own) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = gl + GW * r;
        if (RJ >= 0 && r < RJ) {
          vbuf[buf][i] = 0.0;
          continue;
        }
        const double vi = col[r] * sv;
        vbuf[buf][i] = below(r) ? vi : (diag(r) ? 1.0 : 0.0);
        col[r] = below(r) ? vi : (diag(r) ? beta : col[r]);
      }
      if (gl == 0) {
        taubuf[buf] = tau;
        if (tau_out) tau_out[j] = tau;
      }
    }
  };
  // The block index j / GW is uniform across the wave: one compiled form per
  // block, chosen by a scalar branch, where the look-ahead is unrolled over
  // few slots.
  auto build = [&](int j, double(&col)[R]) {
    if constexpr (S * R <= 16) {
      const int rj = j / GW;
      qr_static_for<R>([&](auto rjc) {
        if (rj == decltype(rjc)::value) build_rows(rjc, j, col);
      });
    } else {
      build_rows(std::integral_constant<int, -1>{}, j, col);
    }
  };
  // whether slot s of this wave holds a column after j (and before nc)
  auto active = [&](int j, int s) {
    const int cw = wave * GPW + NG * s;  // first column of the wave's slot
    return cw + GPW - 1 > j && cw < nc;
  };
  // Reflector j (v, tau) applied to slot s of this wave.
  auto apply = [&](int j, double(&col)[R], int s, const double(&v)[R], double tau) {
    if (!active(j, s)) return;
    double p[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) p[q] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) p[r % NP] += v[r] * col[r];
    double dot = p[0];
#pragma unroll
    for (int q = 1; q < NP; ++q) dot += p[q];
    dot = group_allsum<GW>(dot);
    const int c = grp + NG * s;
    const double w = (c > j && c < nc) ? tau * dot : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) col[r] -= w * v[r];
  };

  if (n > 0 && wave == owner_wave(0)) build(0, a[0]);
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    const int jn = j + 1;
    const bool la = jn < n && wave == owner_wave(jn);
    const int sn = jn / NG;
    auto load_v = [&](double(&v)[R]) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = vbuf[j & 1][gl + GW * r];
    };
    if (la) {
      // the look-ahead is the serial part of the step: let it issue first
      __builtin_amdgcn_s_setprio(2);
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (s == sn) {
          // v and tau in one LDS round trip
          double v[R];
          load_v(v);
          const double tau = taubuf[j & 1];
          apply(j, a[s], s, v, tau);
          build(jn, a[s]);
        }
      __builtin_amdgcn_s_setprio(0);
      // v is read again below rather than kept live through the build
      asm volatile("" ::: "memory");
    }
    // waves with no column after j read nothing
    bool more = false;
#pragma unroll
    for (int s = 0; s < S; ++s) more |= (!la || s != sn) && active(j, s);
    if (more) {
      double v[R];
      load_v(v);
      const double tau = taubuf[j & 1];
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (!la || s != sn) apply(j, a[s], s, v, tau);
    }
  }

  // outputs of the factorisation, and the top n rows to LDS
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int c = grp + NG * s;
    if (c >= nc) continue;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = gl + GW * r;
      if (i >= m) continue;
      if (fact_out && c < n) fact_out[i + (int64_t)c * m] = a[s][r];
      if (i < n) {
        rs[i + c * n] = a[s][r];
        if (Rout && c < n) Rout[i + (int64_t)c * ldr] = i <= c ? a[s][r] : 0.0;
        if (i == c && (a[s][r] == 0.0 || !isfinite(a[s][r]))) s_singular = 1;
      }
    }
  }
  __syncthreads();
  if (s_singular) {
    for (int64_t t = threadIdx.x; t < (int64_t)n * nrhs; t += blockDim.x) {
      const int c = (int)(t / n), i = (int)(t - (int64_t)c * n);
      X[i + (int64_t)c * ldx] = __longlong_as_double(0x7ff8000000000000LL);
    }
    if (threadIdx.x == 0) {
      record_status(status, MS_ERR_SINGULAR);
      if (status2) record_status(status2, MS_ERR_SINGULAR);
    }
    return;
  }
  // n <= m <= GW R, so a wave holds y in (GW R + 63) / 64 registers per lane
  for (int c = wave; c < nrhs; c += NW)
    wave_back_substitute_reg<(GW * R + 63) / 64>(n, rs, n, rs + (int64_t)(n + c) * n,
                                                 X + (int64_t)c * ldx);
}

template <int NW, int GW, int R, int S>
__global__ __launch_bounds__(NW * 64) void k_qr_reg(int m, int n, int nrhs, const double *__restrict__ W,
                                                 int64_t ldw, const double *__restrict__ Bm,
                                                 int64_t ldb, const double *__restrict__ part,
                                                 const float *__restrict__ part32, int nsplit,
                                                 double *__restrict__ X, int64_t ldx,
                                                 double *__restrict__ Rm, int64_t ldr,
                                                 double *__restrict__ tau_out,
                                                 double *__restrict__ fact_out, int *status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ QrShared<GW * R> sh;
  qr_reg_body<NW, GW, R, S>(m, n, nrhs, W, ldw, Bm, ldb, part, part32, nsplit, X, ldx, Rm, ldr,
                            tau_out,
                        fact_out, status, nullptr, reinterpret_cast<double *>(smem_raw), sh);
}

// One workgroup per problem of a batch: Z_p (FP64, k2 x (n + nrhs)) -> X_p.
// first register shape that fits an m x nc system (defined with the shape table)
__host__ __device__ inline int qr_first_shape(int64_t m, int64_t nc);

template <int NW, int GW, int R, int S>
__global__ __launch_bounds__(NW * 64) void k_batch_qr(int count, const ms_problem *__restrict__ P,
                                                   const BatchEntry *__restrict__ E,
                                                   const unsigned char *__restrict__ zarea,
                                                   unsigned char *__restrict__ farea,
                                                   int *__restrict__ pstatus, int *status,
                                                   int64_t lds_doubles, int shape_class) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ QrShared<GW * R> sh;
  const int p = blockIdx.x;
  const BatchEntry &e = E[p];
  if (!e.valid) return;
  const ms_problem &Q = P[p];
  const double *Z = reinterpret_cast<const double *>(zarea + e.z_off);
  const int m = (int)Q.k2, n = (int)Q.n;
  // deterministic mode: one launch per shape, each problem factored by the
  // first shape that fits it alone (the shape fixes the reduction order)
  if (shape_class >= 0 && qr_first_shape(m, e.nc) != shape_class) return;
  // descriptors rewritten after the launch shape was chosen must still fit it
  if (m > GW * R || e.nc > (NW * 64 / GW) * S || (int64_t)n * e.nc > lds_doubles) {
    if (threadIdx.x == 0) {
      record_status(&pstatus[p], MS_ERR_NOMEM);
      record_status(status, MS_ERR_NOMEM);
    }
    return;
  }
  double *fact = batch_ref(e) ? reinterpret_cast<double *>(farea + e.f_off) : nullptr;
  double *tau = fact ? fact + (int64_t)m * n : nullptr;
  qr_reg_body<NW, GW, R, S>(m, n, (int)Q.nrhs, Z, m, Z + (int64_t)n * m, m, nullptr, nullptr, 0, Q.X,
                        Q.ldx, nullptr, 0, tau, fact, &pstatus[p], status,
                        reinterpret_cast<double *>(smem_raw), sh);
}

struct QrRegShape {
  int nw, gw, r, s;  // waves, group width, rows per lane (m <= gw r), slots (nc <= groups s)
};
// the register-resident instantiations, cheapest first.  Sixteen waves: with
// fewer (more slots per group) the column updates of the owning wave lengthen
// every step, which measured slower at every shape tried.
constexpr QrRegShape kQrShapes[] = {
    {16, 16, 1, 1}, {16, 16, 2, 1}, {16, 16, 4, 1}, {16, 16, 2, 2}, {16, 16, 8, 1}, {16, 16, 4, 2},
    {16, 16, 8, 2}, {16, 16, 8, 3}, {16, 32, 8, 2}, {16, 32, 8, 3}, {16, 32, 8, 4}, {16, 32, 8, 5}};
#define MS_QR_SHAPES(X)                                                                \
  X(16, 16, 1, 1) X(16, 16, 2, 1) X(16, 16, 4, 1) X(16, 16, 2, 2) X(16, 16, 8, 1)     \
  X(16, 16, 4, 2) X(16, 16, 8, 2) X(16, 16, 8, 3) X(16, 32, 8, 2) X(16, 32, 8, 3)     \
  X(16, 32, 8, 4) X(16, 32, 8, 5)

static bool shape_fits(const QrRegShape &s, int64_t m, int64_t nc) {
  return s.gw * s.r >= m && (s.nw * 64 / s.gw) * s.s >= nc;
}

// Index in kQrShapes of the first register shape that fits an m x nc system
// (-1: none); the same first-fit rule on the device.
__host__ __device__ inline int qr_first_shape(int64_t m, int64_t nc) {
  int j = 0;
#define MS_QR_FIRST(W_, G_, R_, S_)                                        \
  if ((int64_t)G_ * R_ >= m && (int64_t)(W_ * 64 / G_) * S_ >= nc) return j; \
  ++j;
  MS_QR_SHAPES(MS_QR_FIRST)
#undef MS_QR_FIRST
  return -1;
}

template <int NW, int GW, int R, int S>
static hipError_t launch_qr_reg_t(int64_t m, int64_t n, int64_t nrhs, const double *W,
                                  int64_t ldw, const double *Bm, int64_t ldb, const double *part,
                                  const float *part32, int nsplit, double *X, int64_t ldx,
                                  double *Rm, int64_t ldr,
                                  double *tau_out, double *fact_out, int *status,
                                  hipStream_t st) {
  const size_t lds = (size_t)n * (size_t)(n + nrhs) * sizeof(double);
  hipError_t e = allow_dynamic_lds((const void *)k_qr_reg<NW, GW, R, S>, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_qr_reg<NW, GW, R, S>), dim3(1), dim3(NW * 64), lds, st, (int)m, (int)n,
                     (int)nrhs, W, ldw, Bm, ldb, part, part32, nsplit, X, ldx, Rm, ldr, tau_out,
                     fact_out, status);
  return hipGetLastError();
}

// Returns hipErrorNotSupported when no register-resident shape fits.
bool qr_reg_fits(int64_t m, int64_t n, int64_t nrhs) {
  const int64_t nc = n + nrhs;
  const size_t lds = (size_t)n * (size_t)nc * sizeof(double) + 2 * 256 * 8 + 64;
  if (lds > (size_t)dev_info().lds_per_block) return false;
  for (const QrRegShape &s : kQrShapes)
    if (shape_fits(s, m, nc)) return true;
  return false;
}

hipError_t launch_qr_reg(int64_t m, int64_t n, int64_t nrhs, const double *W, int64_t ldw,
                         const double *Bm, int64_t ldb, const double *part, const float *part32,
                         int nsplit, double *X, int64_t ldx, double *R, int64_t ldr,
                         double *tau_out, double *fact_out, int *status, hipStream_t st) {
  const int64_t nc = n + nrhs;
  if (!qr_reg_fits(m, n, nrhs)) return hipErrorNotSupported;
  for (const QrRegShape &s : kQrShapes) {
    if (!shape_fits(s, m, nc)) continue;
#define MS_QR_CASE(W_, G_, R_, S_)                                                             \
  if (s.nw == W_ && s.gw == G_ && s.r == R_ && s.s == S_)                                      \
    return launch_qr_reg_t<W_, G_, R_, S_>(m, n, nrhs, W, ldw, Bm, ldb, part, part32, nsplit, X, \
                                           ldx, R, ldr, tau_out, fact_out, status, st);
    MS_QR_SHAPES(MS_QR_CASE)
#undef MS_QR_CASE
  }
  return hipErrorNotSupported;
}

// M (m x (n + nrhs)) for the blocked and global-memory paths, then n values
// of tau for the blocked path when the caller keeps none.
size_t qr_workspace_bytes(int64_t m, int64_t n, int64_t nrhs) {
  return ((size_t)m * (size_t)(n + nrhs) + (size_t)n) * sizeof(double);
}

// ------------------------------------------------------------------ blocked QR
// Householder QR of a system too large for one workgroup's registers but with
// at most 1024 rows: [W | Bm] is copied to M (m x nc, ld m) and factored in
// panels of kPanel columns.  A panel kernel (one workgroup; wave jj owns
// panel column jj in registers, lane l rows l + 64 r) computes the panel's
// reflectors in order and leaves them below the diagonal with R on and above
// it, exactly as the unblocked factorisation does; an update kernel applies
// the panel's reflectors, in order, to every later column (one wave per
// column, reflectors staged in LDS), right-hand sides included.  The
// reflectors and the arithmetic per column are those of the unblocked
// algorithm: only the schedule differs.
constexpr int kPanel = 16;

__global__ void k_qrb_load(int m, int n, int nrhs, const double *__restrict__ W, int64_t ldw,
                           const double *__restrict__ Bm, int64_t ldb, double *__restrict__ M) {
  const int64_t total = (int64_t)m * (n + nrhs);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / m), i = (int)(t - (int64_t)c * m);
    M[t] = c < n ? W[i + (int64_t)c * ldw] : Bm[i + (int64_t)(c - n) * ldb];
  }
}

template <int RPL>
__global__ __launch_bounds__(1024) void k_qrb_panel(int m, int n, int j0, double *__restrict__ M,
                                                    double *__restrict__ tau_out) {
  __shared__ double vbuf[2][64 * RPL];
  __shared__ double taubuf[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = min(kPanel, n - j0);
  const int c = j0 + wave;
  double a[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + 64 * r;
    a[r] = (wave < b && i < m) ? M[i + (int64_t)c * m] : 0.0;
  }
  for (int jj = 0; jj < b; ++jj) {
    const int j = j0 + jj, buf = jj & 1;
    if (wave == jj) {
      double p2 = 0.0, av = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i > j && i < m) p2 += a[r] * a[r];
        if (r == (j >> 6)) av = a[r];
      }
      const double xn2 = wave_allsum(p2);
      const double alpha = read_lane(av, j & 63);
      double tau = 0.0, beta = alpha, scal = 0.0;
      if (xn2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + xn2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        const double v = (i > j && i < m) ? a[r] * scal : (i == j ? 1.0 : 0.0);
        vbuf[buf][i] = v;
        if (xn2 != 0.0) a[r] = i > j ? v : (i == j ? beta : a[r]);
      }
      if (lane == 0) {
        taubuf[buf] = tau;
        tau_out[j] = tau;
      }
    }
    __syncthreads();
    const double tau = taubuf[buf];
    if (tau != 0.0 && wave > jj && wave < b) {
      double dot = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) dot += vbuf[buf][lane + 64 * r] * a[r];
      const double w = tau * wave_allsum(dot);
#pragma unroll
      for (int r = 0; r < RPL; ++r) a[r] -= w * vbuf[buf][lane + 64 * r];
    }
  }
  if (wave < b) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      if (i >= j0 && i < m) M[i + (int64_t)c * m] = a[r];
    }
  }
}

// Apply the reflectors of panel [j0, j0 + b) to columns j0 + b + 16 * blockIdx.x
// + wave (< nc).  Dynamic LDS: b * 64 * RPL doubles.
template <int RPL>
__global__ __launch_bounds__(1024) void k_qrb_update(int m, int n, int nc, int j0,
                                                     double *__restrict__ M,
                                                     const double *__restrict__ tau) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *V = reinterpret_cast<double *>(smem_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = min(kPanel, n - j0);
  const int rows = 64 * RPL;
  for (int t = threadIdx.x; t < b * rows; t += blockDim.x) {
    const int jj = t / rows, i = t - jj * rows, j = j0 + jj;
    V[t] = (i > j && i < m) ? M[i + (int64_t)j * m] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = j0 + b + 16 * blockIdx.x + wave;
  if (c >= nc) return;
  double y[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + 64 * r;
    y[r] = i < m ? M[i + (int64_t)c * m] : 0.0;
  }
  for (int jj = 0; jj < b; ++jj) {
    const double tj = tau[j0 + jj];
    if (tj == 0.0) continue;
    const double *v = V + jj * rows;
    double dot = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) dot += v[lane + 64 * r] * y[r];
    const double w = tj * wave_allsum(dot);
#pragma unroll
    for (int r = 0; r < RPL; ++r) y[r] -= w * v[lane + 64 * r];
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + 64 * r;
    if (i >= j0 && i < m) M[i + (int64_t)c * m] = y[r];
  }
}

// Outputs of the blocked factorisation and the back substitution.
__global__ __launch_bounds__(1024) void k_qrb_finish(int m, int n, int nrhs,
                                                     double *__restrict__ M,
                                                     double *__restrict__ X, int64_t ldx,
                                                     double *__restrict__ R, int64_t ldr,
                                                     double *__restrict__ fact_out, int *status) {
  __shared__ int s_singular;
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) s_singular = 0;
  __syncthreads();
  if (fact_out)
    for (int64_t t = tid; t < (int64_t)m * n; t += blockDim.x) fact_out[t] = M[t];
  if (R)
    for (int64_t t = tid; t < (int64_t)n * n; t += blockDim.x) {
      const int c = (int)(t / n), i = (int)(t - (int64_t)c * n);
      R[i + (int64_t)c * ldr] = i <= c ? M[i + (int64_t)c * m] : 0.0;
    }
  for (int i = tid; i < n; i += blockDim.x) {
    const double r = M[i + (int64_t)i * m];
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
    wave_back_substitute(n, M, m, M + (int64_t)(n + c) * m, X + (int64_t)c * ldx);
}

template <int RPL>
static hipError_t launch_qr_blocked_t(int64_t m, int64_t n, int64_t nrhs, const double *W,
                                      int64_t ldw, const double *Bm, int64_t ldb, double *X,
                                      int64_t ldx, double *R, int64_t ldr, double *tau_out,
                                      double *fact_out, double *M, int *status,
                                      hipStream_t st) {
  const int64_t nc = n + nrhs;
  const unsigned lb = (unsigned)std::min<int64_t>((m * nc + 255) / 256, 4096);
  hipLaunchKernelGGL(k_qrb_load, dim3(lb), dim3(256), 0, st, (int)m, (int)n, (int)nrhs, W, ldw,
                     Bm, ldb, M);
  hipError_t e = hipGetLastError();
  const size_t lds = (size_t)kPanel * 64 * RPL * sizeof(double);
  if (e == hipSuccess) e = allow_dynamic_lds((const void *)k_qrb_update<RPL>, (int)lds);
  for (int64_t j0 = 0; j0 < n && e == hipSuccess; j0 += kPanel) {
    hipLaunchKernelGGL(k_qrb_panel<RPL>, dim3(1), dim3(1024), 0, st, (int)m, (int)n, (int)j0, M,
                       tau_out);
    e = hipGetLastError();
    const int64_t rest = nc - std::min<int64_t>(n, j0 + kPanel);
    if (e == hipSuccess && rest > 0) {
      hipLaunchKernelGGL(k_qrb_update<RPL>, dim3((unsigned)((rest + 15) / 16)), dim3(1024), lds,
                         st, (int)m, (int)n, (int)nc, (int)j0, M, (const double *)tau_out);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_qrb_finish, dim3(1), dim3(1024), 0, st, (int)m, (int)n, (int)nrhs, M, X,
                       ldx, R, ldr, fact_out, status);
    e = hipGetLastError();
  }
  return e;
}

// Blocked path for 256 < m <= 1024 (or systems too wide for the register
// kernel); tau_out must be a device array of n doubles.
static hipError_t launch_qr_blocked(int64_t m, int64_t n, int64_t nrhs, const double *W,
                                    int64_t ldw, const double *Bm, int64_t ldb, double *X,
                                    int64_t ldx, double *R, int64_t ldr, double *tau_out,
                                    double *fact_out, double *M, int *status, hipStream_t st) {
  if (m <= 256)
    return launch_qr_blocked_t<4>(m, n, nrhs, W, ldw, Bm, ldb, X, ldx, R, ldr, tau_out, fact_out,
                                  M, status, st);
  if (m <= 512)
    return launch_qr_blocked_t<8>(m, n, nrhs, W, ldw, Bm, ldb, X, ldx, R, ldr, tau_out, fact_out,
                                  M, status, st);
  return launch_qr_blocked_t<16>(m, n, nrhs, W, ldw, Bm, ldb, X, ldx, R, ldr, tau_out, fact_out,
                                 M, status, st);
}

hipError_t launch_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W, int64_t ldw,
                           const double *Bm, int64_t ldb, double *X, int64_t ldx, double *R,
                           int64_t ldr, double *tau_out, double *fact_out, void *qr_ws,
                           int *status, hipStream_t st) {
  hipError_t er = launch_qr_reg(m, n, nrhs, W, ldw, Bm, ldb, nullptr, nullptr, 0, X, ldx, R, ldr,
                                tau_out, fact_out, status, st);
  if (er != hipErrorNotSupported) return er;
  const DevInfo &di = dev_info();
  const size_t bytes = (size_t)m * (size_t)(n + nrhs) * sizeof(double);
  if (bytes + 1024 > (size_t)di.lds_per_block && m <= 1024 && qr_ws) {
    double *M = static_cast<double *>(qr_ws);
    double *tau = tau_out ? tau_out : M + m * (n + nrhs);
    return launch_qr_blocked(m, n, nrhs, W, ldw, Bm, ldb, X, ldx, R, ldr, tau, fact_out, M,
                             status, st);
  }
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

hipError_t launch_batch_qr(int count, int max_k2, int max_n, int max_nc, const ms_problem *P,
                           const BatchEntry *E, const unsigned char *zarea, unsigned char *farea,
                           int *pstatus, int *status, hipStream_t st, int det) {
  const size_t lds = (size_t)max_n * (size_t)max_nc * sizeof(double);
  const int last = qr_first_shape(max_k2, max_nc);
  if (last < 0) return hipErrorNotSupported;
  // default: the one shape that fits the largest problem; deterministic:
  // every shape up to that one, each taking the problems it fits first
  const int first = det ? 0 : last;
  for (int j = first; j <= last; ++j) {
    const QrRegShape &s = kQrShapes[j];
    const int cls = det ? j : -1;
    hipError_t e = hipErrorNotSupported;
#define MS_BQR_CASE(W_, G_, R_, S_)                                                            \
  if (s.nw == W_ && s.gw == G_ && s.r == R_ && s.s == S_) {                                   \
    e = allow_dynamic_lds((const void *)k_batch_qr<W_, G_, R_, S_>, (int)lds);               \
    if (e != hipSuccess) return e;                                                            \
    hipLaunchKernelGGL((k_batch_qr<W_, G_, R_, S_>), dim3(count), dim3(W_ * 64), lds, st,     \
                       count, P, E,                                                           \
                       zarea, farea, pstatus, status, (int64_t)max_n * max_nc, cls);          \
    e = hipGetLastError();                                                                    \
  }
    MS_QR_SHAPES(MS_BQR_CASE)
#undef MS_BQR_CASE
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Refinement of a batch, one workgroup per problem: zr = the G Yr partials
// summed in split order; dx = R^{-1} (Q^T zr)_{0:n} with the reflectors, tau
// and R the first pass kept; X += dx.  One wave per right-hand side, which
// holds its column in registers (lane l rows l + 64 r); the next reflector
// (and, in the back substitution, the next column of R) is loaded while the
// current one is applied.
__global__ __launch_bounds__(64 * kBatchMaxRefineRhs) void k_batch_apply_solve(
    int count, const ms_problem *__restrict__ P, BatchEntry *__restrict__ E,
    const unsigned char *__restrict__ gvarea, const unsigned char *__restrict__ farea,
    int tol_log2) {
  constexpr int RPL = kBatchMaxK2 / 64;
  __shared__ double zb[kBatchMaxK2 * kBatchMaxRefineRhs];
  __shared__ double nrm[2][kBatchMaxRefineRhs];   // per right-hand side: ||dx||^2, ||X||^2
  const int p = blockIdx.x;
  const BatchEntry &e = E[p];
  if (!batch_ref(e)) return;
  const ms_problem &Q = P[p];
  const int m = (int)Q.k2, n = (int)Q.n, nrhs = (int)Q.nrhs;
  if (m > kBatchMaxK2 || nrhs > kBatchMaxRefineRhs) return;  // excluded by the setup
  const int64_t MN = (int64_t)m * nrhs;
  const double *part = reinterpret_cast<const double *>(gvarea + e.gv_off);
  for (int t = threadIdx.x; t < MN; t += blockDim.x) {
    double s = part[t];
    for (int z = 1; z < e.nsplit; ++z) s = s + part[t + (int64_t)z * MN];
    zb[t] = s;
  }
  __syncthreads();
  const double *fact = reinterpret_cast<const double *>(farea + e.f_off);
  const double *tau = fact + (int64_t)m * n;
  const int lane = threadIdx.x & 63, c = threadIdx.x >> 6;
  if (c >= nrhs) {
    // waves without a right-hand side only join the convergence check
    if (tol_log2 > 0) __syncthreads();
    return;
  }
  double y[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + 64 * r;
    y[r] = i < m ? zb[c * m + i] : 0.0;
  }
  // y <- Q^T y, reflector j: v_i = fact[i, j] below the diagonal, 1 on it
  auto load_v = [&](int j, double v[RPL]) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      v[r] = (i > j && i < m) ? fact[i + (int64_t)j * m] : (i == j ? 1.0 : 0.0);
    }
  };
  double vn[RPL], tn = n > 0 ? tau[0] : 0.0;
  if (n > 0) load_v(0, vn);
  for (int j = 0; j < n; ++j) {
    double v[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) v[r] = vn[r];
    const double tj = tn;
    if (j + 1 < n) {
      load_v(j + 1, vn);
      tn = tau[j + 1];
    }
    double dot = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) dot += v[r] * y[r];
    const double w = tj * wave_allsum(dot);
#pragma unroll
    for (int r = 0; r < RPL; ++r) y[r] -= w * v[r];
  }
  // R dx = y[0:n): column i of R is fact[0:i, i] (on and above the diagonal)
  auto load_r = [&](int i, double col[RPL]) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int t = lane + 64 * r;
      col[r] = t <= i ? fact[t + (int64_t)i * m] : 0.0;
    }
  };
  double rn[RPL];
  double dx2 = 0.0, x2 = 0.0;   // lane 0: sums over this right-hand side
  if (n > 0) load_r(n - 1, rn);
  for (int i = n - 1; i >= 0; --i) {
    double col[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) col[r] = rn[r];
    if (i > 0) load_r(i - 1, rn);
    double yl = 0.0, dl = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r)
      if (r == (i >> 6)) {
        yl = y[r];
        dl = col[r];
      }
    const double xi = read_lane(yl, i & 63) / read_lane(dl, i & 63);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int t = lane + 64 * r;
      if (t < i) y[r] -= col[r] * xi;
    }
    if (lane == 0) {
      const double xn = Q.X[i + (int64_t)c * Q.ldx] + xi;
      Q.X[i + (int64_t)c * Q.ldx] = xn;
      dx2 += xi * xi;
      x2 += xn * xn;
    }
  }
  if (tol_log2 > 0) {
    // converged when ||dx||_F <= 2^-tol ||X||_F: the later steps skip the
    // problem (its entry's refine flag cleared; the setup of the next
    // launch sets it again)
    if (lane == 0) {
      nrm[0][c] = dx2;
      nrm[1][c] = x2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double sd = 0.0, sx = 0.0;
      for (int q = 0; q < nrhs; ++q) {
        sd += nrm[0][q];
        sx += nrm[1][q];
      }
      if (sd <= ldexp(sx, -2 * tol_log2)) E[p].refine = 0;
    }
  }
}

hipError_t launch_batch_apply_solve(int count, const ms_problem *P, BatchEntry *E,
                                    const unsigned char *gvarea, const unsigned char *farea,
                                    int *pstatus, int *status, hipStream_t st, int tol_log2) {
  (void)pstatus;
  (void)status;
  hipLaunchKernelGGL(k_batch_apply_solve, dim3(count), dim3(64 * kBatchMaxRefineRhs), 0, st,
                     count, P, E, gvarea, farea, tol_log2);
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

// The same for m <= 64 * RPL with each right-hand side in one wave's
// registers (lane l rows l + 64 r); the next reflector, and in the back
// substitution the next column of R, are loaded while the current one is
// applied.  Bm is left unchanged.
template <int RPL>
__global__ __launch_bounds__(512) void k_qr_apply_solve_reg(int m, int n, int nrhs,
                                                             const double *__restrict__ fact,
                                                             const double *__restrict__ tau,
                                                             const double *__restrict__ Bm,
                                                             double *__restrict__ X, int64_t ldx,
                                                             int *status) {
  __shared__ int s_singular;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
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
  auto load_v = [&](int j, double v[RPL]) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      v[r] = (i > j && i < m) ? fact[i + (int64_t)j * m] : (i == j ? 1.0 : 0.0);
    }
  };
  auto load_r = [&](int i, double col[RPL]) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int t = lane + 64 * r;
      col[r] = t <= i ? fact[t + (int64_t)i * m] : 0.0;
    }
  };
  for (int c = wave; c < nrhs; c += nw) {
    double y[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      y[r] = i < m ? Bm[i + (int64_t)c * m] : 0.0;
    }
    double vn[RPL], tn = tau[0];
    load_v(0, vn);
    for (int j = 0; j < n; ++j) {
      double v[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[r] = vn[r];
      const double tj = tn;
      if (j + 1 < n) {
        load_v(j + 1, vn);
        tn = tau[j + 1];
      }
      if (tj == 0.0) continue;
      double dot = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) dot += v[r] * y[r];
      const double w = tj * wave_allsum(dot);
#pragma unroll
      for (int r = 0; r < RPL; ++r) y[r] -= w * v[r];
    }
    double rn[RPL];
    load_r(n - 1, rn);
    for (int i = n - 1; i >= 0; --i) {
      double col[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) col[r] = rn[r];
      if (i > 0) load_r(i - 1, rn);
      double yl = 0.0, dl = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        if (r == (i >> 6)) {
          yl = y[r];
          dl = col[r];
        }
      const double xi = read_lane(yl, i & 63) / read_lane(dl, i & 63);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int t = lane + 64 * r;
        if (t < i) y[r] -= col[r] * xi;
      }
      if (lane == 0) X[i + (int64_t)c * ldx] = xi;
    }
  }
}

hipError_t launch_qr_apply_solve(int64_t m, int64_t n, int64_t nrhs, const double *fact,
                                 const double *tau, double *Bm, double *X, int64_t ldx,
                                 int *status, hipStream_t st) {
  if (n < 1 || nrhs < 1) return hipSuccess;
  const unsigned threads = (unsigned)(64 * std::min<int64_t>(nrhs, 8));
#define MS_AS_CASE(R_)                                                                         \
  if (m <= 64 * R_) {                                                                         \
    hipLaunchKernelGGL(k_qr_apply_solve_reg<R_>, dim3(1), dim3(threads), 0, st, (int)m, (int)n, \
                       (int)nrhs, fact, tau, (const double *)Bm, X, ldx, status);              \
    return hipGetLastError();                                                                 \
  }
  MS_AS_CASE(1)
  MS_AS_CASE(2)
  MS_AS_CASE(4)
  MS_AS_CASE(8)
  MS_AS_CASE(16)
#undef MS_AS_CASE
  hipLaunchKernelGGL(k_qr_apply_solve, dim3(1), dim3(1024), 0, st, (int)m, (int)n, (int)nrhs,
                     fact, tau, Bm, X, ldx, status);
  return hipGetLastError();
}

}  // namespace ms
