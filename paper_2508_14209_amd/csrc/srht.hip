// srht.hip -- the SRHT S = k^{-1/2} P H_m D (Sec. 5) of a column-major m x
// ncols operand X, and through it the second stage of the Count + SRHT
// multisketch (Sec. 8's future-work variant).
//
// H_m (m the smallest power of two >= the rows of X, X padded with zero
// rows) factors over blocks of B = 8192 rows: H_m = (H_{m/B} (x) I_B)
// (I_{m/B} (x) H_B).  Row r of H_m D X is therefore
//   sum over blocks q of (-1)^{popcount((r >> 13) AND q)} (H_B D_q X_q)[r mod B],
// so one pass over X suffices: each workgroup transforms one block of one
// column in place (D, then the 13 butterfly stages of H_B), keeps only the k
// sampled rows with their block sign, and the per-block values are summed
// over blocks in block order afterwards.  Only the sampled rows leave the
// workgroup: X is read once and nothing of its size is written.
//
// Inside a block each of 256 threads holds 32 elements in registers.  The
// butterfly stages on the 5 index bits a thread holds run in registers; the
// 13 bits are covered by three such sets (bits 8-12, 0-4, 5-7) with two
// exchanges through LDS in between, instead of one LDS round trip per stage
// as in the stage-by-stage FWHT (Alg. 3 processes two bits per stage).
// Blocks of fewer than 8192 rows (m < 8192) use a plain stage-by-stage LDS
// transform.
#include "ms_internal.h"

namespace ms {

namespace {

constexpr int kLogB = 13;
constexpr int kB = 1 << kLogB;
constexpr int kThreads = 256;      // 32 elements per thread
constexpr int kPer = kB / kThreads;
constexpr int kRCache = 1024;      // sampled row indices kept in LDS

// LDS slot of block element e: one pad slot per 32 elements keeps the three
// exchange patterns free of bank conflicts beyond the 64-bit pairs
__device__ __forceinline__ int pad(int e) { return e + (e >> 5); }

__device__ __forceinline__ double block_sign(int64_t r, int64_t q) {
  return (__popcll((uint64_t)(r >> kLogB) & (uint64_t)q) & 1) ? -1.0 : 1.0;
}

// butterflies of the stages on the register-index bits in [lo, lo + nb)
template <int LO, int NB>
__device__ __forceinline__ void reg_stages(double (&x)[kPer]) {
#pragma unroll
  for (int b = LO; b < LO + NB; ++b)
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (!(u & (1 << b))) {
        const double a = x[u], c = x[u | (1 << b)];
        x[u] = a + c;
        x[u | (1 << b)] = a - c;
      }
}

// Persistent: workgroup g takes items g, g + grid, ... (item = c nblk + q:
// block q of column c), and loads the next item's 32 values per thread into
// registers before it transforms the current one, so a block's HBM reads
// overlap the previous block's butterflies and LDS exchanges.  out: with one
// block, Y (scaled); else part[(q ncols + c) k + j] (unscaled, summed by
// k_srht_reduce).
// Element maps of the three register phases (t: thread, u: register):
//   phase 1  e = (u & 3) | t << 2 | (u >> 2) << 10        bits 0,1,10,11,12 in registers
//   phase 2  e = (t & 3) | u << 2 | (t >> 2) << 7         bits 2..6
//   phase 3  e = (t & 127) | (u & 7) << 7 | (t >> 7) << 10 | (u >> 3) << 11   bits 7,8,9
// Phase 1 gives each thread 8 groups of 4 consecutive rows: one 32-byte load
// and one 4-byte sign word per group (16 load instructions per thread), so a
// wave stays well under its limit of 63 outstanding loads and the next
// block's loads are all in flight while the current block is transformed.
// With the one pad slot per 32 elements, every exchange reaches each LDS
// bank pair at most twice per 64 lanes.
// pad(e_k(t, u)) = p_k(t) + c_k(u): a per-thread base plus a compile-time
// offset (at most 59 KB, inside the LDS instruction's immediate), so each
// exchange keeps one address register instead of 32.
__device__ __forceinline__ int p1(int t) { return 4 * t + (t >> 3); }
constexpr int c1(int u) { return (u & 3) + 1056 * (u >> 2); }
__device__ __forceinline__ int p2(int t) { return (t & 3) + 132 * (t >> 2); }
constexpr int c2(int u) { return 4 * u + (u >> 3); }
__device__ __forceinline__ int p3(int t) { return (t & 127) + ((t & 127) >> 5) + 1056 * (t >> 7); }
constexpr int c3(int u) { return 132 * (u & 7) + 2112 * (u >> 3); }
__device__ __forceinline__ int e1(int t, int u) { return (u & 3) | (t << 2) | ((u >> 2) << 10); }

typedef double dv4e __attribute__((ext_vector_type(4), aligned(8)));
typedef float fv4e __attribute__((ext_vector_type(4), aligned(4)));
template <typename T>
struct V4;
template <>
struct V4<double> {
  typedef dv4e type;
};
template <>
struct V4<float> {
  typedef fv4e type;
};

// Raw loads of one item (block q of column c) in the phase-1 map; nothing
// here uses the data, so the loads stay in flight.  Full blocks (all 8192
// rows inside X) with a 4-byte aligned dsign take vector loads; the ragged
// last block reads clamped rows one by one (zeroed by srht_signed).
template <typename TX>
__device__ __forceinline__ void srht_load(int64_t item, int nblk, int64_t mx,
                                          const TX *__restrict__ X, int64_t ldx,
                                          const int8_t *__restrict__ dsign, bool svec, int t,
                                          TX (&xa)[kPer], uint32_t (&sw)[kPer / 4]) {
  const int64_t q = item % nblk, c = item / nblk;
  const int64_t base = q * kB;
  const TX *xc = X + c * ldx;
  if (svec && base + kB <= mx) {
#pragma unroll
    for (int g = 0; g < kPer / 4; ++g) {
      const int64_t i = base + e1(t, 4 * g);
      const typename V4<TX>::type v = gload((const typename V4<TX>::type *)(xc + i));
#pragma unroll
      for (int r = 0; r < 4; ++r) xa[4 * g + r] = v[r];
      sw[g] = gload((const uint32_t *)(dsign + i));
    }
  } else {
#pragma unroll
    for (int g = 0; g < kPer / 4; ++g) {
      uint32_t w = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = base + e1(t, 4 * g + r);
        const int64_t ic = i < mx ? i : mx - 1;
        xa[4 * g + r] = gload(xc + ic);
        w |= (uint32_t)(uint8_t)gload(dsign + ic) << (8 * r);
      }
      sw[g] = w;
    }
  }
}

// D applied to the loaded values (FP64), rows past mx zeroed; a sign other
// than +-1 sets bad.
template <typename TX>
__device__ __forceinline__ void srht_signed(int64_t base, int64_t mx, int t,
                                            const TX (&xa)[kPer], const uint32_t (&sw)[kPer / 4],
                                            double (&x)[kPer], bool &bad) {
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const bool in = base + e1(t, u) < mx;
    const int8_t sg = (int8_t)(sw[u >> 2] >> (8 * (u & 3)));
    bad |= in & !(sg == 1 || sg == -1);
    const double a = (double)xa[u];
    x[u] = in ? (sg < 0 ? -a : a) : 0.0;
  }
}

template <typename TX>
__global__ __launch_bounds__(kThreads) void k_srht_block(int64_t mx, int ncols, int k, int nblk,
                                                         const TX *__restrict__ X, int64_t ldx,
                                                         const int8_t *__restrict__ dsign,
                                                         const int32_t *__restrict__ r,
                                                         int64_t m, double scale,
                                                         double *__restrict__ out, int64_t ldo,
                                                         int *status) {
  __shared__ double lds[kB + kB / 32];
  // the sampled rows, the same for every item: read from LDS, so that the
  // sampling does not wait behind the next item's loads
  __shared__ int32_t rs[kRCache];
  const int t = threadIdx.x;
  const int64_t items = (int64_t)nblk * ncols;
  const bool svec = (reinterpret_cast<uintptr_t>(dsign) & 3) == 0;
  for (int j = t; j < k && j < kRCache; j += kThreads) rs[j] = gload(r + j);
  bool bad = false;
  TX xa[kPer];
  uint32_t sw[kPer / 4];
  int64_t item = blockIdx.x;
  if (item < items) srht_load(item, nblk, mx, X, ldx, dsign, svec, t, xa, sw);
  for (; item < items; item += gridDim.x) {
    const int64_t q = item % nblk, c = item / nblk;
    double x[kPer];
    srht_signed(q * kB, mx, t, xa, sw, x, bad);
    const int64_t next = item + gridDim.x;
    if (next < items) srht_load(next, nblk, mx, X, ldx, dsign, svec, t, xa, sw);
    reg_stages<0, 5>(x);  // bits 0, 1, 10, 11, 12
    __syncthreads();      // the previous item's sampling reads are done
    double *const l1 = lds + p1(t);
    double *const l2 = lds + p2(t);
    double *const l3 = lds + p3(t);
#pragma unroll
    for (int u = 0; u < kPer; ++u) l1[c1(u)] = x[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) x[u] = l2[c2(u)];
    reg_stages<0, 5>(x);  // bits 2..6
#pragma unroll
    for (int u = 0; u < kPer; ++u) l2[c2(u)] = x[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) x[u] = l3[c3(u)];
    reg_stages<0, 3>(x);  // bits 7, 8, 9
#pragma unroll
    for (int u = 0; u < kPer; ++u) l3[c3(u)] = x[u];
    __syncthreads();
    // the sampled rows of this block's share
    auto sample = [&](int j, int32_t rj) {
      const bool ok = rj >= 0 && (int64_t)rj < m;
      bad |= !ok;
      const double v = ok ? block_sign(rj, q) * lds[pad(rj & (kB - 1))] : 0.0;
      if (nblk == 1)
        out[j + c * ldo] = v * scale;
      else
        out[(q * ncols + c) * k + j] = v;
    };
    // two uniform paths: a global load on the same path as the LDS read
    // would make the LDS path wait for every outstanding load too
    if (k <= kRCache) {
      for (int j = t; j < k; j += kThreads) sample(j, rs[j]);
    } else {
      for (int j = t; j < k; j += kThreads) sample(j, gload(r + j));
    }
  }
  if (bad) record_status(status, MS_ERR_RANGE);
}

// m < 8192: one workgroup per column, the whole transform in LDS, one
// butterfly stage at a time.
template <typename TX>
__global__ __launch_bounds__(kThreads) void k_srht_small(int64_t mx, int logm, int k,
                                                         const TX *__restrict__ X, int64_t ldx,
                                                         const int8_t *__restrict__ dsign,
                                                         const int32_t *__restrict__ r,
                                                         double scale, double *__restrict__ Y,
                                                         int64_t ldy, int *status) {
  __shared__ double lds[kB];
  const int t = threadIdx.x;
  const int c = blockIdx.x;
  const int m = 1 << logm;
  const TX *xc = X + (int64_t)c * ldx;
  bool bad = false;
  for (int i = t; i < m; i += kThreads) {
    double v = 0.0;
    if (i < mx) {
      const int8_t sg = gload(dsign + i);
      bad |= !(sg == 1 || sg == -1);
      const double a = (double)gload(xc + i);
      v = sg < 0 ? -a : a;
    }
    lds[i] = v;
  }
  __syncthreads();
  for (int b = 0; b < logm; ++b) {
    for (int p = t; p < m / 2; p += kThreads) {
      const int i0 = ((p >> b) << (b + 1)) | (p & ((1 << b) - 1));
      const int i1 = i0 | (1 << b);
      const double a = lds[i0], cc = lds[i1];
      lds[i0] = a + cc;
      lds[i1] = a - cc;
    }
    __syncthreads();
  }
  for (int j = t; j < k; j += kThreads) {
    const int32_t rj = gload(r + j);
    const bool ok = rj >= 0 && rj < m;
    bad |= !ok;
    Y[j + (int64_t)c * ldy] = ok ? lds[rj] * scale : 0.0;
  }
  if (bad) record_status(status, MS_ERR_RANGE);
}

// Y[j][c] = scale * the sum over blocks q of part[(q ncols + c) k + j]: a
// workgroup takes 64 consecutive outputs (one column); wave w sums the
// blocks of its contiguous share in ascending order (four interleaved
// running sums, added pairwise), and the 16 waves' sums are added in wave
// order -- a fixed association, so repeated calls give the same bits.
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(64 * kRedWaves) void k_srht_reduce(int ncols, int k, int nblk,
                                                                const double *__restrict__ part,
                                                                double scale,
                                                                double *__restrict__ Y,
                                                                int64_t ldy) {
  __shared__ double sh[kRedWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tiles = (k + 63) / 64;
  const int c = blockIdx.x / tiles;
  const int j = (blockIdx.x % tiles) * 64 + lane;
  const int q0 = (int)((int64_t)nblk * w / kRedWaves), q1 = (int)((int64_t)nblk * (w + 1) / kRedWaves);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < k) {
    const double *p = part + (int64_t)c * k + j;
    const int64_t step = (int64_t)ncols * k;
    int q = q0;
    for (; q + 4 <= q1; q += 4)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += p[(int64_t)(q + u) * step];
    for (int u = 0; q < q1; ++q, ++u) s[u] += p[(int64_t)q * step];
  }
  sh[w][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (w == 0 && j < k) {
    double t = 0.0;
    for (int v = 0; v < kRedWaves; ++v) t += sh[v][lane];
    Y[j + (int64_t)c * ldy] = t * scale;
  }
}

}  // namespace

int64_t srht_padded_rows(int64_t mx) {
  int64_t m = 1;
  while (m < mx) m *= 2;
  return m;
}

size_t srht_workspace_bytes(int64_t mx, int64_t ncols, int64_t k) {
  const int64_t m = srht_padded_rows(mx);
  const int64_t nblk = m > kB ? m / kB : 1;
  return nblk > 1 ? (size_t)nblk * ncols * k * 8 : 0;
}

template <typename TX>
hipError_t launch_srht(int64_t mx, int64_t ncols, int64_t k, const TX *X, int64_t ldx,
                       const int8_t *dsign, const int32_t *r, double *Y, int64_t ldy, void *part,
                       int *status, hipStream_t st) {
  if (mx < 1 || ncols < 1 || k < 1) return hipSuccess;
  if (ncols > 65535) return hipErrorInvalidValue;
  const int64_t m = srht_padded_rows(mx);
  const double scale = 1.0 / sqrt((double)k);
  if (m < kB) {
    int logm = 0;
    while ((int64_t)1 << logm < m) ++logm;
    hipLaunchKernelGGL((k_srht_small<TX>), dim3((unsigned)ncols), dim3(kThreads), 0, st, mx, logm,
                       (int)k, X, ldx, dsign, r, scale, Y, ldy, status);
    return hipGetLastError();
  }
  const int64_t nblk = m / kB;
  // persistent grid: two workgroups per CU (the LDS of a block allows two)
  const int64_t items = nblk * ncols;
  const unsigned grid = (unsigned)std::min<int64_t>(items, 2 * (int64_t)dev_info().cus);
  if (nblk == 1) {
    hipLaunchKernelGGL((k_srht_block<TX>), dim3(grid), dim3(kThreads), 0, st, mx, (int)ncols,
                       (int)k, 1, X, ldx, dsign, r, m, scale, Y, ldy, status);
    return hipGetLastError();
  }
  if (!part) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_srht_block<TX>), dim3(grid), dim3(kThreads), 0, st, mx, (int)ncols,
                     (int)k, (int)nblk, X, ldx, dsign, r, m, scale, static_cast<double *>(part),
                     (int64_t)0, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned rb = (unsigned)(ncols * ((k + 63) / 64));
  hipLaunchKernelGGL(k_srht_reduce, dim3(rb), dim3(64 * kRedWaves), 0, st, (int)ncols, (int)k,
                     (int)nblk, static_cast<const double *>(part), scale, Y, ldy);
  return hipGetLastError();
}
template hipError_t launch_srht<double>(int64_t, int64_t, int64_t, const double *, int64_t,
                                        const int8_t *, const int32_t *, double *, int64_t, void *,
                                        int *, hipStream_t);
template hipError_t launch_srht<float>(int64_t, int64_t, int64_t, const float *, int64_t,
                                       const int8_t *, const int32_t *, double *, int64_t, void *,
                                       int *, hipStream_t);

}  // namespace ms
