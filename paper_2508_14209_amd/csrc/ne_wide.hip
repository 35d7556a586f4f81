// ne_wide.hip -- the normal equations (Sec. 6.3's comparator) and the
// Cholesky stage of rand_cholQR (Alg. 5) for wide problems: n up to 256
// columns with up to 16 right-hand sides (n + nrhs <= 272).
//
//   W = V^T V with V = [X | B] (d x nc), X = A (normal equations) or
//   X = Q0 = A R0^{-1} (rand_cholQR), FP64; R1 = chol(W_XX); y = R1^{-T} W_XB;
//   x = R1^{-1} y.
//
// The Gram pass is a tall product, bound by the FP64 matrix cores
// (n (n + 1) + 2 n nrhs flops per row; 2 nc^2 flops of a full product).
// Its upper 16 x 16 tiles are handed out as tasks of up to 2 x 4 tiles
// (tile rows it0, it0 + 1; tile columns jt0 .. jt0 + 3), so a wave keeps 8
// accumulator tiles and 6 operand fragments in registers.  Workgroups of
// four waves take one task and one chunk of rows; the waves of a workgroup
// split the chunk's 16-row slabs, their sums are added in wave order and the
// workgroup's partial goes to its chunk's slice of a partial buffer; an
// ordered pass then adds the chunks.  All tasks of a chunk run on one die
// (workgroup g on die g % 8), so the chunk's rows come from HBM once and the
// tasks' re-reads hit that die's L2.
//
// The factorisation and solves run in one workgroup by 64 x 64 blocks, the
// Gram matrix's upper part factored in place.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double dvec4e __attribute__((ext_vector_type(4), aligned(8)));
typedef float fvec4e __attribute__((ext_vector_type(4), aligned(4)));
template <typename T>
struct Four4;
template <>
struct Four4<double> {
  typedef dvec4e type;
};
template <>
struct Four4<float> {
  typedef fvec4e type;
};

constexpr int kGwWaves = 4;      // waves per Gram workgroup
constexpr int kSolveN = 256;     // order of the register-resident factorisation

__device__ __forceinline__ v4d mma64w(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Rows row .. row + 3 of a column (all inside it), promoted to FP64.
template <typename T>
__device__ __forceinline__ v4d rows4(const T *p, int64_t row) {
  const typename Four4<T>::type x = gload((const typename Four4<T>::type *)(p + row));
  return v4d{(double)x[0], (double)x[1], (double)x[2], (double)x[3]};
}
// Same, zero past row d.
template <typename T>
__device__ __forceinline__ v4d rows4_guard(const T *p, int64_t row, int64_t d) {
  v4d v = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (row + r < d) v[r] = (double)gload(p + row + r);
  return v;
}

// Task t of the upper tile triangle of an NT x NT tile grid: tile rows
// it0 = 0, 2, 4, ..., and for each, tile columns jt0 = it0, it0 + 4, ...
__host__ __device__ inline void wide_task(int NT, int t, int &it0, int &jt0) {
  for (int a = 0; a < NT; a += 2) {
    const int cnt = (NT - a + 3) / 4;
    if (t < cnt) {
      it0 = a;
      jt0 = a + 4 * t;
      return;
    }
    t -= cnt;
  }
  it0 = jt0 = NT;
}

__host__ __device__ inline int wide_ntasks(int NT) {
  int c = 0;
  for (int a = 0; a < NT; a += 2) c += (NT - a + 3) / 4;
  return c;
}

// The column c of V = [X | B] (null past nc).
template <typename TX, typename TB>
struct VCols {
  const TX *X;
  int64_t ldx;
  const TB *B;
  int64_t ldb;
  int nx, nc;
};

template <typename TX, typename TB>
__global__ __launch_bounds__(64 * kGwWaves) void k_gram_wide(int64_t d, VCols<TX, TB> v, int NT,
                                                             int ntasks, int nchunks, int xcds,
                                                             double *__restrict__ part,
                                                             int64_t pstride, int np) {
  __shared__ double wsum[8 * 256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int g = blockIdx.x;
  const int x = g % xcds, idx = g / xcds;
  const int task = idx % ntasks;
  const int chunk = (idx / ntasks) * xcds + x;
  if (chunk >= nchunks) return;
  int it0, jt0;
  wide_task(NT, task, it0, jt0);
  const bool diag = it0 == jt0;
  // which of the 2 x 4 tiles exist (it <= jt, both inside the grid): uniform
  bool ok[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) ok[i][j] = it0 + i < NT && jt0 + j < NT && it0 + i <= jt0 + j;

  // column pointers of this lane's fragments: tile rows (I) and columns (J);
  // columns past nc read column 0 and are masked
  auto colp = [&](int c, bool &valid) -> const void * {
    valid = c < v.nc;
    if (!valid) c = 0;
    return c < v.nx ? (const void *)(v.X + (int64_t)c * v.ldx)
                    : (const void *)(v.B + (int64_t)(c - v.nx) * v.ldb);
  };
  const void *ip[2], *jp[4];
  bool iv[2], jv[4], ix[2], jx[4];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int c = 16 * min(it0 + i, NT - 1) + li;
    ip[i] = colp(c, iv[i]);
    ix[i] = (iv[i] ? c : 0) < v.nx;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 16 * min(jt0 + j, NT - 1) + li;
    jp[j] = colp(c, jv[j]);
    jx[j] = (jv[j] ? c : 0) < v.nx;
  }
  auto load = [&](const void *p, bool isx, int64_t row, bool full) -> v4d {
    if (isx)
      return full ? rows4(static_cast<const TX *>(p), row)
                  : rows4_guard(static_cast<const TX *>(p), row, d);
    return full ? rows4(static_cast<const TB *>(p), row)
                : rows4_guard(static_cast<const TB *>(p), row, d);
  };

  v4d acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t nslab = (d + 15) >> 4;
  const int64_t s0 = nslab * chunk / nchunks, s1 = nslab * (chunk + 1) / nchunks;
  const int64_t nfull = d >> 4;
  for (int64_t sl = s0 + wave; sl < s1; sl += kGwWaves) {
    const int64_t rr = sl * 16 + 4 * lk;
    const bool full = sl < nfull;
    v4d fj[4], fi[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      fj[j] = load(jp[j], jx[j], rr, full);
      if (!jv[j]) fj[j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    if (diag) {
      fi[0] = fj[0];
      fi[1] = fj[1];
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fi[i] = load(ip[i], ix[i], rr, full);
        if (!iv[i]) fi[i] = v4d{0.0, 0.0, 0.0, 0.0};
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (ok[i][j])
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j] = mma64w(fi[i][r], fj[j][r], acc[i][j]);
  }
  // the waves' sums in wave order; the last wave writes the chunk's partial
  double *P = part + (int64_t)chunk * pstride;
  for (int wv = 0; wv < kGwWaves; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (ok[i][j])
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int si = (i * 4 + j) * 256 + lane * 4 + r;
              const double val = wv == 0 ? acc[i][j][r] : wsum[si] + acc[i][j][r];
              if (wv == kGwWaves - 1)
                P[(int64_t)(16 * (it0 + i) + lk + 4 * r) * np + 16 * (jt0 + j) + li] = val;
              else
                wsum[si] = val;
            }
    }
    if (wv < kGwWaves - 1) __syncthreads();
  }
}

// W[e] = sum over chunks (in chunk order, four interleaved running sums
// added pairwise) of the partials' entry e, for the entries of upper tiles.
__global__ void k_gram_wide_reduce(int nchunks, int NT, int np, const double *__restrict__ part,
                                   int64_t pstride, double *__restrict__ W) {
  const int64_t total = (int64_t)np * np;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / np), col = (int)(e - (int64_t)row * np);
    if ((row >> 4) > (col >> 4)) continue;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int c = 0;
    for (; c + 3 < nchunks; c += 4)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += part[(int64_t)(c + u) * pstride + e];
    for (int u = 0; c < nchunks; ++c, ++u) s[u] += part[(int64_t)c * pstride + e];
    W[e] = (s[0] + s[1]) + (s[2] + s[3]);
  }
}

// W_XX = R1^T R1 in place by a blocked right-looking Cholesky with 64 x 64
// blocks (per block: the diagonal block by one wave with a column per lane
// in registers; the block row by forward substitution; the trailing upper
// part by 64 x 64 chunk products staged in LDS), then R1^T y = W_XB and
// R1 x = y by blocks (a wave solves the block's triangle, every thread
// updates the remaining rows), and for rand_cholQR (fact non-null: R0 on and
// above the diagonal of the k2 x n QR factors, ld ldf) x = R0^{-1} x by the
// same blocked back substitution.  W is row-major with leading dimension np
// (upper part read and overwritten).  Rout (optional): R1, or R1 R0 for
// rand_cholQR, n x n column-major, zeros below the diagonal.
constexpr int kCsB = 64;    // block order
constexpr int kCsL = 65;    // LDS row stride of a block
constexpr int kCsT = 256;   // threads

__device__ __forceinline__ double rd_lane(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// element (i, j) of an upper-triangular factor: R1 in W (row-major, np) or
// R0 in fact (column-major, ldf)
struct TriRef {
  const double *p;
  int64_t ld;
  bool rowmajor;
  __device__ double operator()(int i, int j) const {
    return rowmajor ? p[(int64_t)i * ld + j] : p[i + (int64_t)j * ld];
  }
};

// z (LDS, z[c * 256 + i], nrhs columns) := U^{-1} z for upper-triangular U
// of order n (blocked backward substitution; all 256 threads call it).
__device__ void back_solve(const TriRef &U, int n, int nrhs, double *z) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int nb = (n + kCsB - 1) / kCsB;
  for (int kb = nb - 1; kb >= 0; --kb) {
    const int r0 = kCsB * kb, m = min(kCsB, n - r0);
    if (tid < 64 && lane < nrhs) {
      for (int t = m - 1; t >= 0; --t) {
        const double xt = z[lane * 256 + r0 + t] / U(r0 + t, r0 + t);
        z[lane * 256 + r0 + t] = xt;
        for (int i = 0; i < t; ++i) z[lane * 256 + r0 + i] -= U(r0 + i, r0 + t) * xt;
      }
    }
    __syncthreads();
    for (int i = tid; i < r0; i += kCsT) {
      for (int c = 0; c < nrhs; ++c) {
        double s = 0.0;
        for (int t = 0; t < m; ++t) s += U(i, r0 + t) * z[c * 256 + r0 + t];
        z[c * 256 + i] -= s;
      }
    }
    __syncthreads();
  }
}

// (a) Diagonal block kb of the blocked Cholesky: one wave, lane l holding
// column l of the block's upper part; R_kk is written back in place.  A
// breakdown sets *bad (every later launch then returns at once).  Block 0
// clears *bad first.
__global__ __launch_bounds__(64) void k_chol_diag(int n, int np, int kb, double *__restrict__ W,
                                                  int *__restrict__ bad) {
  __shared__ double rb[kCsB * kCsL];
  const int lane = threadIdx.x;
  if (kb == 0) {
    if (lane == 0) *bad = 0;
  } else if (*bad) {
    return;
  }
  const int r0 = kCsB * kb, m = min(kCsB, n - r0);
  double g[kCsB];
#pragma unroll
  for (int i = 0; i < kCsB; ++i)
    g[i] = (i < m && lane < m) ? (i <= lane ? W[(int64_t)(r0 + i) * np + r0 + lane] : 0.0)
                               : (i == lane ? 1.0 : 0.0);
  bool fail = false;
#pragma unroll
  for (int j = 0; j < kCsB; ++j) {
    const double djj = rd_lane(g[j], j);
    if (!(djj > 0.0) || !isfinite(djj)) {
      fail = true;
      break;
    }
    const double rjj = sqrt(djj);
    const double rl = lane > j ? g[j] / rjj : (lane == j ? rjj : 0.0);
    g[j] = rl;
    rb[j * kCsL + lane] = rl;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int i = j + 1; i < kCsB; ++i) g[i] -= rb[j * kCsL + i] * rl;
  }
  if (fail) {
    if (lane == 0) *bad = 1;
    return;
  }
  if (lane < m)
#pragma unroll
    for (int i = 0; i < kCsB; ++i)
      if (i < m && i <= lane) W[(int64_t)(r0 + i) * np + r0 + lane] = g[i];
}

// (b) Block row kb (columns c >= r0 + 64: R_kk^T x = W[r0:r0+m, c], by
// 64-column chunks staged in LDS, one column per lane of wave 0), then the
// trailing update W[i][c] -= sum_t R[r0+t][i] R[r0+t][c] for
// r0 + 64 <= i <= c < n by 64 x 64 chunk products staged in LDS.
__global__ __launch_bounds__(kCsT) void k_chol_panel(int n, int np, int kb,
                                                     double *__restrict__ W,
                                                     const int *__restrict__ bad) {
  __shared__ double dk[kCsB * kCsL];
  __shared__ double pn[kCsB * kCsL];
  if (*bad) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r0 = kCsB * kb, m = min(kCsB, n - r0);
  for (int t = tid; t < kCsB * kCsB; t += kCsT) {
    const int i = t >> 6, j = t & 63;
    dk[i * kCsL + j] = (i < m && j < m) ? (i <= j ? W[(int64_t)(r0 + i) * np + r0 + j] : 0.0)
                                        : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int c0 = r0 + kCsB; c0 < n; c0 += kCsB) {
    for (int t = tid; t < kCsB * kCsB; t += kCsT) {
      const int i = t >> 6, j = t & 63;
      pn[i * kCsL + j] = (i < m && c0 + j < n) ? W[(int64_t)(r0 + i) * np + c0 + j] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      for (int i = 0; i < m; ++i) {
        double s = pn[i * kCsL + lane];
        for (int q = 0; q < i; ++q) s -= dk[q * kCsL + i] * pn[q * kCsL + lane];
        pn[i * kCsL + lane] = s / dk[i * kCsL + i];
      }
    }
    __syncthreads();
    for (int t = tid; t < kCsB * kCsB; t += kCsT) {
      const int i = t >> 6, j = t & 63;
      if (i < m && c0 + j < n) W[(int64_t)(r0 + i) * np + c0 + j] = pn[i * kCsL + j];
    }
    __syncthreads();
  }
  for (int cc = r0 + kCsB; cc < n; cc += kCsB) {
    for (int t = tid; t < kCsB * kCsB; t += kCsT) {
      const int tt = t >> 6, j = t & 63;
      pn[tt * kCsL + j] = (tt < m && cc + j < n) ? W[(int64_t)(r0 + tt) * np + cc + j] : 0.0;
    }
    for (int ic = r0 + kCsB; ic <= cc; ic += kCsB) {
      __syncthreads();
      for (int t = tid; t < kCsB * kCsB; t += kCsT) {
        const int tt = t >> 6, j = t & 63;
        dk[tt * kCsL + j] = (tt < m && ic + j < n) ? W[(int64_t)(r0 + tt) * np + ic + j] : 0.0;
      }
      __syncthreads();
      const int il = tid >> 2;
      double acc[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = 0.0;
      for (int t = 0; t < m; ++t) {
        const double a = dk[t * kCsL + il];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] += a * pn[t * kCsL + (tid & 3) + 4 * u];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = ic + il, c = cc + (tid & 3) + 4 * u;
        if (i <= c && c < n) W[(int64_t)i * np + c] -= acc[u];
      }
    }
    __syncthreads();
  }
}

// (c) The solves: R1^T y = W_XB (blocked forward substitution), R1 x = y,
// and for rand_cholQR (fact non-null) x = R0^{-1} x; X, and Rout (R1, or
// R1 R0 for rand_cholQR) when asked for.  After a breakdown: X = NaN and
// MS_ERR_SINGULAR.
__global__ __launch_bounds__(kCsT) void k_chol_solves(int n, int nrhs, int np,
                                                      const double *__restrict__ W,
                                                      const double *__restrict__ fact,
                                                      int64_t ldf, double *__restrict__ X,
                                                      int64_t ldx, double *__restrict__ Rout,
                                                      int64_t ldr, const int *__restrict__ bad,
                                                      int *status) {
  __shared__ double zs[16 * 256];
  const int tid = threadIdx.x, lane = tid & 63;
  if (*bad) {
    for (int t = tid; t < n * nrhs; t += kCsT) {
      const int c = t / n, i = t - c * n;
      X[i + (int64_t)c * ldx] = __longlong_as_double(0x7ff8000000000000LL);
    }
    if (tid == 0) record_status(status, MS_ERR_SINGULAR);
    return;
  }
  for (int t = tid; t < 16 * 256; t += kCsT) {
    const int c = t >> 8, i = t & 255;
    zs[t] = (c < nrhs && i < n) ? W[(int64_t)i * np + n + c] : 0.0;
  }
  __syncthreads();
  const int nb = (n + kCsB - 1) / kCsB;
  for (int kb = 0; kb < nb; ++kb) {
    const int r0 = kCsB * kb, m = min(kCsB, n - r0);
    if (tid < 64 && lane < nrhs) {
      for (int t = 0; t < m; ++t) {
        const double yt = zs[lane * 256 + r0 + t] / W[(int64_t)(r0 + t) * np + r0 + t];
        zs[lane * 256 + r0 + t] = yt;
        for (int i = t + 1; i < m; ++i)
          zs[lane * 256 + r0 + i] -= W[(int64_t)(r0 + t) * np + r0 + i] * yt;
      }
    }
    __syncthreads();
    for (int i = r0 + m + tid; i < n; i += kCsT) {
      for (int c = 0; c < nrhs; ++c) {
        double s = 0.0;
        for (int t = 0; t < m; ++t) s += W[(int64_t)(r0 + t) * np + i] * zs[c * 256 + r0 + t];
        zs[c * 256 + i] -= s;
      }
    }
    __syncthreads();
  }
  back_solve(TriRef{W, np, true}, n, nrhs, zs);
  if (fact) back_solve(TriRef{fact, ldf, false}, n, nrhs, zs);
  for (int t = tid; t < n * nrhs; t += kCsT) {
    const int c = t / n, i = t - c * n;
    X[i + (int64_t)c * ldx] = zs[c * 256 + i];
  }
  if (Rout) {
    for (int t = tid; t < n * n; t += kCsT) {
      const int j = t / n, i = t - j * n;
      double v = 0.0;
      if (i <= j) {
        if (fact)
          for (int q = i; q <= j; ++q) v += W[(int64_t)i * np + q] * fact[q + (int64_t)j * ldf];
        else
          v = W[(int64_t)i * np + j];
      }
      Rout[i + (int64_t)j * ldr] = v;
    }
  }
}

int wide_nt(int nc) { return (nc + 15) / 16; }

}  // namespace

// Chunks of rows of the wide Gram pass: about two workgroups of four waves
// per compute unit in all, a multiple of the die count, at least 64 slabs
// of 16 rows per chunk.
int gram_wide_chunks(int64_t d, int nc) {
  const DevInfo &di = dev_info();
  const int xcds = di.xcds > 0 ? di.xcds : 1;
  const int ntasks = wide_ntasks(wide_nt(nc));
  int64_t c = std::max<int64_t>(1, (int64_t)2 * di.cus / ntasks);
  c = std::min<int64_t>(c, std::max<int64_t>(1, ((d + 15) / 16) / 64));
  c = (c + xcds - 1) / xcds * xcds;
  return (int)std::min<int64_t>(c, 4096);
}

size_t gram_wide_partial_bytes(int64_t d, int nc) {
  const int np = 16 * wide_nt(nc);
  return (size_t)gram_wide_chunks(d, nc) * np * np * sizeof(double);
}

size_t gram_wide_w_bytes(int nc) {
  const int np = 16 * wide_nt(nc);
  return (size_t)np * np * sizeof(double);
}

template <typename TX, typename TB>
hipError_t launch_gram_wide(int64_t d, int nx, int nc, const TX *X, int64_t ldx, const TB *B,
                            int64_t ldb, double *part, double *W, hipStream_t st) {
  if (nc < 1 || nc > kWideMaxCols || nx < 0 || nx > nc) return hipErrorInvalidValue;
  const DevInfo &di = dev_info();
  const int xcds = di.xcds > 0 ? di.xcds : 1;
  const int NT = wide_nt(nc), np = 16 * NT;
  const int ntasks = wide_ntasks(NT);
  const int nchunks = gram_wide_chunks(d, nc);
  const int64_t pstride = (int64_t)np * np;
  VCols<TX, TB> v{X, ldx, B, ldb, nx, nc};
  const unsigned grid = (unsigned)((int64_t)nchunks * ntasks);
  hipLaunchKernelGGL((k_gram_wide<TX, TB>), dim3(grid), dim3(64 * kGwWaves), 0, st, d, v, NT,
                     ntasks, nchunks, xcds, part, pstride, np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned rb = (unsigned)std::min<int64_t>((pstride + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gram_wide_reduce, dim3(rb), dim3(256), 0, st, nchunks, NT, np, part,
                     pstride, W);
  return hipGetLastError();
}
template hipError_t launch_gram_wide<double, double>(int64_t, int, int, const double *, int64_t,
                                                     const double *, int64_t, double *, double *,
                                                     hipStream_t);
template hipError_t launch_gram_wide<float, float>(int64_t, int, int, const float *, int64_t,
                                                   const float *, int64_t, double *, double *,
                                                   hipStream_t);
template hipError_t launch_gram_wide<double, float>(int64_t, int, int, const double *, int64_t,
                                                    const float *, int64_t, double *, double *,
                                                    hipStream_t);

hipError_t launch_chol_solve_wide(int n, int nrhs, int nc, double *W, const double *fact,
                                  int64_t ldf, double *X, int64_t ldx, double *R, int64_t ldr,
                                  int *bad, int *status, hipStream_t st) {
  if (n < 1 || n > kSolveN || nrhs < 0 || nrhs > 16 || n + nrhs > nc) return hipErrorInvalidValue;
  const int np = 16 * wide_nt(nc);
  const int nb = (n + kCsB - 1) / kCsB;
  for (int kb = 0; kb < nb; ++kb) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, n, np, kb, W, bad);
    if (kb + 1 < nb)
      hipLaunchKernelGGL(k_chol_panel, dim3(1), dim3(kCsT), 0, st, n, np, kb, W, (const int *)bad);
  }
  hipLaunchKernelGGL(k_chol_solves, dim3(1), dim3(kCsT), 0, st, n, nrhs, np, (const double *)W,
                     fact, ldf, X, ldx, R, ldr, (const int *)bad, status);
  return hipGetLastError();
}

}  // namespace ms
