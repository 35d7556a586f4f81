// plan_blocked.hip -- the sketch plan (bucket counts, their exclusive scan,
// the rows of every bucket in ascending row order) by blocks of rows, for
// k <= 16384 buckets: every count and cursor lives in LDS, and no global
// atomic is issued.
//
//   1. per block of 4096 rows: a histogram of its buckets in LDS, written
//      out as one row of a blocks x k count table;
//   2. per bucket: the exclusive prefix of its counts over the blocks (the
//      first slot each block's rows of that bucket take within the bucket)
//      and the bucket's total;
//   3. the exclusive scan of the totals (bucket offsets);
//   4. per block: its rows sorted by (bucket, row) in LDS (counting
//      placement and a per-bucket insertion sort; a bitonic network over
//      the 4096 keys when a bucket is long), written to offset[bucket] +
//      prefix[block][bucket] + rank.
// Within a bucket, rows of earlier blocks come first and each block's rows
// ascend: the stable counting sort, with no per-bucket sorting pass.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

constexpr int kPbRows = 4096;  // rows per block
constexpr int kPbT = 1024;     // threads
constexpr int64_t kPbMaxK = MS_SORTED_BLOCKED_MAX_K;

// 1. LDS histogram of block b's buckets, stored as row b of cnt_tab (k
// ints); rows with h outside [0, k) are left out and reported.
__global__ __launch_bounds__(kPbT) void k_pb_hist(int64_t d, int k, const int32_t *__restrict__ h,
                                                  int32_t *__restrict__ tab, int *status) {
  extern __shared__ int32_t lc[];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  for (int m = tid; m < k; m += kPbT) lc[m] = 0;
  __syncthreads();
  const int64_t r0 = b * kPbRows, r1 = min(d, r0 + kPbRows);
  bool bad = false;
#pragma unroll 4
  for (int64_t i = r0 + tid; i < r1; i += kPbT) {
    const int32_t m = h[i];
    if ((uint32_t)m < (uint32_t)k)
      atomicAdd(&lc[m], 1);
    else
      bad = true;
  }
  if (bad) record_status(status, MS_ERR_RANGE);
  __syncthreads();
  for (int m = tid; m < k; m += kPbT) tab[b * k + m] = lc[m];
}

// 2. Column prefix over the blocks: 64 buckets per workgroup (a lane per
// bucket), the 16 waves splitting the blocks into contiguous ranges; tab
// becomes the exclusive prefix, cnt the totals.
__global__ __launch_bounds__(kPbT) void k_pb_colscan(int64_t nblk, int k, int32_t *__restrict__ tab,
                                                     int32_t *__restrict__ cnt) {
  __shared__ int32_t ws[16][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = blockIdx.x * 64 + lane;
  const int64_t b0 = nblk * w / 16, b1 = nblk * (w + 1) / 16;
  // (the block loops unrolled so that many of their independent loads are
  // in flight at once)
  int32_t s = 0;
  if (m < k) {
#pragma unroll 16
    for (int64_t b = b0; b < b1; ++b) s += tab[b * k + m];
  }
  ws[w][lane] = s;
  __syncthreads();
  int32_t run = 0;
  for (int v = 0; v < w; ++v) run += ws[v][lane];
  if (m < k) {
#pragma unroll 16
    for (int64_t b = b0; b < b1; ++b) {
      const int32_t c = tab[b * k + m];
      tab[b * k + m] = run;
      run += c;
    }
    if (w == 15) cnt[m] = run;
  }
}

// 3. Exclusive scan of the bucket totals into off (k + 1 entries) and the
// cursors, by one workgroup (16 entries per thread and pass).
__global__ __launch_bounds__(kPbT) void k_pb_scan(int k, const int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ off,
                                                  int32_t *__restrict__ cursor) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < k; base += 16 * kPbT) {
    int32_t v[16], loc = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int m = base + tid * 16 + q;
      v[q] = m < k ? cnt[m] : 0;
      loc += v[q];
    }
    int32_t incl = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t x = __shfl_up(incl, o, 64);
      if (lane >= o) incl += x;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t run = carry_s + incl - loc;
    for (int u = 0; u < w; ++u) run += wsum[u];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int m = base + tid * 16 + q;
      if (m < k) {
        off[m] = run;
        if (cursor) cursor[m] = run;
      }
      run += v[q];
    }
    __syncthreads();
    if (tid == kPbT - 1) carry_s = run;
    __syncthreads();
  }
  if (tid == 0) off[k] = carry_s;
}

// 4. Block b's rows sorted by (bucket, row) in LDS -- key = bucket << 12 |
// row offset, the sign in bit 31, absent or invalid rows last -- by counting
// (each key placed at its bucket's next slot, then each bucket's keys put in
// row order; a block with a bucket of more than kPbMaxRun rows uses a
// bitonic network instead), then each valid row written to off[bucket] +
// prefix[block][bucket] + its rank within the bucket here.
constexpr uint32_t kPbKeyMask = 0x7fffffffu;
constexpr int kPbMaxRun = 64;   // longest bucket the insertion sort takes
__global__ __launch_bounds__(kPbT) void k_pb_place(int64_t d, int k, const int32_t *__restrict__ h,
                                                   const int8_t *__restrict__ s,
                                                   const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ tab,
                                                   uint32_t *__restrict__ sperm) {
  extern __shared__ __align__(16) int32_t sm[];
  int32_t *lstart = sm;                                          // k
  // kPbRows keys, 16-byte aligned (the sort reads and writes four at a time)
  uint32_t *key = reinterpret_cast<uint32_t *>(sm + ((k + 3) & ~3));
  __shared__ int32_t wsum[16];
  __shared__ int s_long;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * kPbRows, r1 = min(d, r0 + kPbRows);
  for (int m = tid; m < k; m += kPbT) lstart[m] = 0;
  if (tid == 0) s_long = 0;
  __syncthreads();
  uint32_t kvr[kPbRows / kPbT];
#pragma unroll
  for (int jj = 0; jj < kPbRows / kPbT; ++jj) {
    const int q = tid + jj * kPbT;
    const int64_t i = r0 + q;
    uint32_t kv = kPbKeyMask;
    if (i < r1) {
      const int32_t m = h[i];
      if ((uint32_t)m < (uint32_t)k) {
        atomicAdd(&lstart[m], 1);
        kv = ((uint32_t)m << 12) | (uint32_t)q | ((s != nullptr && s[i] < 0) ? kSignBit : 0u);
      }
    }
    kvr[jj] = kv;
    key[q] = kv;
  }
  __syncthreads();
  // exclusive scan of the local counts (thread t owns a contiguous range)
  const int per = (k + kPbT - 1) / kPbT;
  int32_t loc = 0;
  for (int q = 0; q < per; ++q) {
    const int m = tid * per + q;
    if (m < k) {
      loc += lstart[m];
      if (lstart[m] > kPbMaxRun) atomicOr(&s_long, 1);
    }
  }
  int32_t incl = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int32_t run = incl - loc;
  for (int v = 0; v < w; ++v) run += wsum[v];
  const bool longrun = s_long != 0;
  __syncthreads();
  for (int q = 0; q < per; ++q) {
    const int m = tid * per + q;
    if (m < k) {
      const int32_t c = lstart[m];
      lstart[m] = run;
      run += c;
    }
  }
  static_assert(kPbRows == 4096 && kPbT == 1024, "sort4096_lds shape");
  __syncthreads();
  if (longrun) {
    // a bucket too long for the insertion sort below: the bitonic network
    // (sign bit ignored); lstart keeps each bucket's start
    sort4096_lds(key);
  } else {
    // counting placement: each valid key at its bucket's next slot (equal
    // buckets in arrival order), lstart becoming each bucket's end, then
    // every bucket's few keys put in row order by one thread; the slots past
    // the valid keys hold padding
#pragma unroll
    for (int jj = 0; jj < kPbRows / kPbT; ++jj) key[tid + jj * kPbT] = kPbKeyMask;
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kPbRows / kPbT; ++jj) {
      const uint32_t kv = kvr[jj];
      if ((kv & kPbKeyMask) != kPbKeyMask) key[atomicAdd(&lstart[(kv & kPbKeyMask) >> 12], 1)] = kv;
    }
    __syncthreads();
    for (int m = tid; m < k; m += kPbT) {
      const int b1 = lstart[m], b0 = m > 0 ? lstart[m - 1] : 0;
      for (int i = b0 + 1; i < b1; ++i) {
        const uint32_t x = key[i];
        int jx = i;
        while (jx > b0 && (key[jx - 1] & kPbKeyMask) > (x & kPbKeyMask)) {
          key[jx] = key[jx - 1];
          --jx;
        }
        key[jx] = x;
      }
    }
    __syncthreads();
  }
  for (int p = tid; p < kPbRows; p += kPbT) {
    const uint32_t kv = key[p];
    if ((kv & kPbKeyMask) == kPbKeyMask) continue;
    const int m = (int)((kv & kPbKeyMask) >> 12);
    // the bucket's first slot in the block: its start (network) or the end
    // of the bucket before it (counting placement)
    const int st = longrun ? lstart[m] : (m > 0 ? lstart[m - 1] : 0);
    const int64_t pos = (int64_t)off[m] + tab[b * k + m] + (p - st);
    sperm[pos] = (uint32_t)(r0 + (kv & 0xfffu)) | (kv & kSignBit);
  }
}

// The deterministic fold (one thread per bucket and column, the bucket's
// rows in ascending order from +0.0: bit-identical to Alg. 2 read
// sequentially), eight rows' loads issued ahead of their dependent adds.
// Launched over a few columns at a time, so the columns being gathered from
// stay in the 256 MB Infinity Cache while their buckets are folded.
template <typename T>
__global__ __launch_bounds__(256) void k_cs_sorted_cols(int64_t k, Cols<T> cols, int c0,
                                                        const int32_t *__restrict__ off,
                                                        const uint32_t *__restrict__ sperm,
                                                        T *__restrict__ Y, int64_t ldy) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = c0 + (int)blockIdx.y;
  if (b >= k) return;
  const T *cp = c < cols.n_a ? cols.A + (int64_t)c * cols.lda
                             : cols.B + (int64_t)(c - cols.n_a) * cols.ldb;
  const int32_t j0 = off[b], j1 = off[b + 1];
  T y = T(0);
  int32_t j = j0;
  for (; j + 8 <= j1; j += 8) {
    uint32_t e[8];
    T a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = sperm[j + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = gload(cp + (e[u] & kIdxMask));
#pragma unroll
    for (int u = 0; u < 8; ++u) y = y + apply_sign(a[u], e[u]);
  }
  for (; j < j1; ++j) {
    const uint32_t e = sperm[j];
    y = y + apply_sign(gload(cp + (e & kIdxMask)), e);
  }
  Y[b + (int64_t)c * ldy] = y;
}

}  // namespace

size_t plan_blocked_bytes(int64_t d, int64_t k) {
  if (k < 1 || k > kPbMaxK || d < 1 || d > 0x7ffffffe) return 0;
  const int64_t nblk = (d + kPbRows - 1) / kPbRows;
  return align_up((size_t)nblk * k * 4);
}

hipError_t launch_plan_blocked(int64_t d, int64_t k, const int32_t *h, const int8_t *s,
                               int32_t *cnt, int32_t *off, int32_t *cursor, void *tab_ws,
                               uint32_t *sperm, int *status, hipStream_t st) {
  if (!plan_blocked_bytes(d, k)) return hipErrorInvalidValue;
  const int64_t nblk = (d + kPbRows - 1) / kPbRows;
  int32_t *tab = static_cast<int32_t *>(tab_ws);
  const int kk = (int)k;
  size_t lds1 = (size_t)k * 4;
  hipError_t e = allow_dynamic_lds((const void *)k_pb_hist, (int)lds1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pb_hist, dim3((unsigned)nblk), dim3(kPbT), lds1, st, d, kk, h, tab, status);
  hipLaunchKernelGGL(k_pb_colscan, dim3((unsigned)((k + 63) / 64)), dim3(kPbT), 0, st, nblk, kk,
                     tab, cnt);
  hipLaunchKernelGGL(k_pb_scan, dim3(1), dim3(kPbT), 0, st, kk, (const int32_t *)cnt, off, cursor);
  const size_t lds4 = (size_t)((k + 3) & ~3) * 4 + (size_t)kPbRows * 4;
  e = allow_dynamic_lds((const void *)k_pb_place, (int)lds4);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pb_place, dim3((unsigned)nblk), dim3(kPbT), lds4, st, d, kk, h, s,
                     (const int32_t *)off, (const int32_t *)tab, sperm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cs_sorted_cols(int64_t k, const Cols<T> &c, const int32_t *off,
                                 const uint32_t *sperm, T *Y, int64_t ldy, hipStream_t st) {
  constexpr int kCols = 8;  // columns per launch
  for (int c0 = 0; c0 < c.ncols; c0 += kCols) {
    const int nc = std::min(kCols, c.ncols - c0);
    hipLaunchKernelGGL(k_cs_sorted_cols<T>, dim3((unsigned)((k + 255) / 256), (unsigned)nc),
                       dim3(256), 0, st, k, c, c0, off, sperm, Y, ldy);
  }
  return hipGetLastError();
}
template hipError_t launch_cs_sorted_cols<double>(int64_t, const Cols<double> &, const int32_t *,
                                                  const uint32_t *, double *, int64_t,
                                                  hipStream_t);
template hipError_t launch_cs_sorted_cols<float>(int64_t, const Cols<float> &, const int32_t *,
                                                 const uint32_t *, float *, int64_t, hipStream_t);

}  // namespace ms
