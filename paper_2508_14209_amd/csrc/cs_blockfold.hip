// cs_blockfold.hip -- the deterministic CountSketch (MS_CS_SORTED): every
// bucket sum of Y = C [A | B] (Def. 3, Eq. (2)) folded from +0.0 in ascending
// row order, bit-identical to the sequential loop over the rows of Alg. 2.
//
// Keys (one pass, per block of 4096 rows): each row of the block as the key
// bucket << 12 | row within the block | sign << 31, the block's keys sorted by
// (bucket, row) in LDS with a bitonic network and stored in that order.  A row
// whose bucket is outside [0, k) or whose sign is not +-1 is reported and
// keyed past every bucket.
//
// Fold: one workgroup per (column, bucket range) walks the blocks in order
// with its buckets' sums resident in LDS.  Per block it stages the column's
// 4096 values and the block's sorted keys in LDS (both loaded into registers
// one block ahead, with coalesced loads), and every run of equal buckets in
// the block is folded by one thread, in ascending row order, into that
// bucket's sum.  Per bucket the additions therefore happen in ascending row
// order over the whole column -- the order of the sequential loop -- while A
// is read in its stored order instead of gathered in bucket order.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

typedef uint32_t bf_u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBfRows = 4096;               // rows per block (12 bits of the key)
constexpr int kBfT = 1024;                  // threads
constexpr uint32_t kBfKeyMask = 0x7fffffffu;  // the (bucket, row) part of a key
constexpr uint32_t kBfPad = 0x7fffffffu;    // sorts last; its bucket field exceeds every k
constexpr int64_t kBfMaxK = (int64_t)1 << 19;  // bucket field: bits 12..30
constexpr int kBfMaxParts = 32;
static_assert(kBfRows == 4096 && kBfT == 1024, "the key sort (sort4096_lds) takes 4096 keys on 1024 threads");

__device__ __forceinline__ uint32_t bf_bucket(uint32_t key) { return (key & kBfKeyMask) >> 12; }

// Thread t keys rows 4t .. 4t + 3 of the block (q = row within the block):
// one 16-byte load of h and one 4-byte load of s when the four rows exist
// and the arrays are aligned for it (vec), else four guarded loads.
__device__ __forceinline__ void bf_make_keys(int64_t d, int64_t k, const int32_t *__restrict__ h,
                                             const int8_t *__restrict__ s, int64_t r0, bool vec,
                                             uint32_t (&v)[4], bool &bad) {
  const int q0 = 4 * threadIdx.x;
  const int64_t i0 = r0 + q0;
  int32_t m[4];
  int8_t sg[4];
  if (vec && i0 + 4 <= d) {
    typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
    const i32x4 hm = gload(reinterpret_cast<const i32x4 *>(h + i0));
    const int sw = gload(reinterpret_cast<const int *>(s + i0));
#pragma unroll
    for (int e = 0; e < 4; ++e) m[e] = hm[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) sg[e] = (int8_t)(sw >> (8 * e));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool in = i0 + e < d;
      m[e] = in ? gload(h + i0 + e) : -1;
      sg[e] = in ? gload(s + i0 + e) : (int8_t)1;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t kv = kBfPad;
    if (i0 + e < d) {
      const bool ok = ((int64_t)(uint32_t)m[e] < k) & (m[e] >= 0) & ((sg[e] == 1) | (sg[e] == -1));
      bad |= !ok;
      if (ok) kv = ((uint32_t)m[e] << 12) | (uint32_t)(q0 + e) | (sg[e] < 0 ? kSignBit : 0u);
    }
    v[e] = kv;
  }
}

__global__ __launch_bounds__(kBfT) void k_bf_keys(int64_t d, int k, const int32_t *__restrict__ h,
                                                  const int8_t *__restrict__ s,
                                                  uint32_t *__restrict__ keys, int *status) {
  __shared__ __align__(16) uint32_t key[kBfRows];
  const int64_t r0 = (int64_t)blockIdx.x * kBfRows;
  const bool vec = (((uintptr_t)h & 15) | ((uintptr_t)s & 3)) == 0;
  bool bad = false;
  uint32_t v[4];
  bf_make_keys(d, k, h, s, r0, vec, v, bad);
  if (bad) record_status(status, MS_ERR_RANGE);
  // sort the 4096 keys by their (bucket, row) part, store them from registers
  sort4096_regs(v, key);
  *reinterpret_cast<uint4 *>(keys + r0 + 4 * threadIdx.x) = make_uint4(v[0], v[1], v[2], v[3]);
}

// The same keys for k <= kBfCountMaxK, sorted by counting instead of by a
// network: bucket counts in LDS (the padding keys counted as bucket k), an
// exclusive scan, each key placed at its bucket's next free slot (an LDS
// atomic, so equal buckets land in arrival order), then every bucket's few
// keys put in row order by one thread (insertion sort), which makes the
// result the same ascending (bucket, row) order as the network's.  A block
// with a bucket of more than kBfCountMaxRun rows falls back to the network.
constexpr int kBfCountMaxK = 16384;
constexpr int kBfCountMaxRun = 64;

size_t bf_count_lds(int64_t k) { return (size_t)(k + 1 + 3) / 4 * 16 + (size_t)kBfRows * 4; }

__global__ __launch_bounds__(kBfT) void k_bf_keys_count(int64_t d, int k,
                                                        const int32_t *__restrict__ h,
                                                        const int8_t *__restrict__ s,
                                                        uint32_t *__restrict__ keys, int *status) {
  extern __shared__ __align__(16) uint32_t bsm[];
  __shared__ uint32_t wsum[kBfT / 64];
  __shared__ int s_long;
  uint32_t *cnt = bsm;                              // k + 1 counters
  uint32_t *key = bsm + (k + 1 + 3) / 4 * 4;        // kBfRows keys, 16-byte aligned
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * kBfRows;
  const bool vec = (((uintptr_t)h & 15) | ((uintptr_t)s & 3)) == 0;
  for (int m = tid; m <= k; m += kBfT) cnt[m] = 0;
  if (tid == 0) s_long = 0;
  bool bad = false;
  uint32_t v[4];
  bf_make_keys(d, k, h, s, r0, vec, v, bad);
  if (bad) record_status(status, MS_ERR_RANGE);
  auto bucket_of = [&](uint32_t kv) { return min(bf_bucket(kv), (uint32_t)k); };
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) atomicAdd(&cnt[bucket_of(v[e])], 1u);
  __syncthreads();
  // exclusive scan of the k + 1 counts, thread t owning a contiguous range
  const int per = (k + 1 + kBfT - 1) / kBfT;
  uint32_t loc = 0;
  for (int q = 0; q < per; ++q) {
    const int m = tid * per + q;
    if (m <= k) {
      loc += cnt[m];
      if (cnt[m] > (uint32_t)kBfCountMaxRun && m < k) atomicOr(&s_long, 1);
    }
  }
  uint32_t incl = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  const bool longrun = s_long != 0;
  if (longrun) {
    // a bucket too long for the insertion sort: the network
    sort4096_regs(v, key);
    *reinterpret_cast<uint4 *>(keys + r0 + 4 * tid) = make_uint4(v[0], v[1], v[2], v[3]);
    return;
  }
  uint32_t run = incl - loc;
  for (int u = 0; u < w; ++u) run += wsum[u];
  for (int q = 0; q < per; ++q) {
    const int m = tid * per + q;
    if (m <= k) {
      const uint32_t c = cnt[m];
      cnt[m] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 4; ++e) key[atomicAdd(&cnt[bucket_of(v[e])], 1u)] = v[e];
  __syncthreads();
  // cnt[m] is now the end of bucket m, cnt[m - 1] its start
  for (int m = tid; m < k; m += kBfT) {
    const uint32_t b1 = cnt[m], b0 = m > 0 ? cnt[m - 1] : 0u;
    for (uint32_t i = b0 + 1; i < b1; ++i) {
      const uint32_t x = key[i];
      uint32_t j = i;
      while (j > b0 && (key[j - 1] & kBfKeyMask) > (x & kBfKeyMask)) {
        key[j] = key[j - 1];
        --j;
      }
      key[j] = x;
    }
  }
  __syncthreads();
  *reinterpret_cast<uint4 *>(keys + r0 + 4 * tid) = *reinterpret_cast<const uint4 *>(key + 4 * tid);
}

template <typename T>
__device__ __forceinline__ const T *bf_col(const Cols<T> &c, int j) {
  return j < c.n_a ? c.A + (int64_t)j * c.lda : c.B + (int64_t)(j - c.n_a) * c.ldb;
}

// Fold buckets [m0, m1) of one column col (d rows) into acc (LDS, zero on
// entry; slot m - m0) over the blocks in order; stage and lkey: LDS for one
// block's values and keys (two blocks' when DB: the next block is staged while
// the current one is folded, one barrier per block instead of two).  Thread t loads rows 4t .. 4t + 3 of a block (its
// values and keys) into registers kBfAhead blocks before the block is folded,
// so that a block's loads are in flight while the blocks before it are
// folded.  Ends with the workgroup synchronised.
constexpr int kBfAhead = 4;

template <typename T, bool DB = false>
__device__ __forceinline__ void bf_fold_column(int64_t d, const T *__restrict__ col,
                                               const uint32_t *__restrict__ keys, uint32_t m0,
                                               uint32_t m1, T *acc, T *stage, uint32_t *lkey) {
  const int tid = threadIdx.x;
  const int64_t nblk = (d + kBfRows - 1) / kBfRows;
  typedef T T4 __attribute__((ext_vector_type(4)));
  T4 v[kBfAhead];
  bf_u32x4 kv[kBfAhead];
  // the column's 4-row groups are vector-aligned when its start is
  const bool vec = ((uintptr_t)col & (4 * sizeof(T) - 1)) == 0;
  // block b (past the last block: the last one again, never used) into set j
  auto fetch = [&](int j, int64_t b) {
    const int64_t r = min(b, nblk - 1) * kBfRows + 4 * tid;
    if (vec && r + 4 <= d) {
      v[j] = gload(reinterpret_cast<const T4 *>(col + r));
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[j][q] = gload(col + min(r + q, d - 1));   // rows past d: padding keys
    }
    kv[j] = gload(reinterpret_cast<const bf_u32x4 *>(keys + r));
  };
  auto put = [&](int j, T *sg, uint32_t *kg) {
    *reinterpret_cast<T4 *>(sg + 4 * tid) = v[j];
    *reinterpret_cast<bf_u32x4 *>(kg + 4 * tid) = kv[j];
  };
  // fold the block staged in sg (values) and kg (sorted keys)
  auto fold = [&](const T *sg, const uint32_t *kg) {
    // this thread's four positions 4t .. 4t + 3 and the key before them;
    // the reads of all four runs' sums and first values are issued
    // together, a run inside the four positions is folded in registers,
    // and a run that goes on past them continues from LDS
    const int p0 = 4 * tid;
    const bf_u32x4 k4 = *reinterpret_cast<const bf_u32x4 *>(kg + p0);
    const uint32_t kprev = p0 > 0 ? kg[p0 - 1] : kBfPad;
    uint32_t kq[5] = {kprev, k4[0], k4[1], k4[2], k4[3]};
    bool start[4];
    uint32_t mq[4];
    T a[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      mq[q] = bf_bucket(kq[q + 1]);
      start[q] = mq[q] >= m0 && mq[q] < m1 && bf_bucket(kq[q]) != mq[q];
      a[q] = start[q] ? acc[mq[q] - m0] : T(0);
      x[q] = start[q] ? sg[kq[q + 1] & (kBfRows - 1)] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!start[q]) continue;
      T s = a[q] + apply_sign(x[q], kq[q + 1]);
      // the run's next rows among this thread's positions (static indices)
      bool more = true;
#pragma unroll
      for (int r = q + 1; r < 4; ++r) {
        if (more && bf_bucket(kq[r + 1]) == mq[q])
          s = s + apply_sign(sg[kq[r + 1] & (kBfRows - 1)], kq[r + 1]);
        else
          more = false;
      }
      if (more) {   // the run may go on into the next threads' positions
        // four keys per LDS read; their values are read together once the
        // first of them is known to continue the run, then added in order
        for (int g = p0 + 4; g < kBfRows; g += 4) {
          const bf_u32x4 kn = *reinterpret_cast<const bf_u32x4 *>(kg + g);
          if (bf_bucket(kn[0]) != mq[q]) break;
          T xn[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) xn[e] = sg[kn[e] & (kBfRows - 1)];
          bool cont = true;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (cont && bf_bucket(kn[e]) == mq[q])
              s = s + apply_sign(xn[e], kn[e]);
            else
              cont = false;
          }
          if (!cont) break;
        }
      }
      acc[mq[q] - m0] = s;
    }
  };
#pragma unroll
  for (int j = 0; j < kBfAhead; ++j) fetch(j, j);
  if constexpr (DB) {
    // two staging buffers: block b + 1 is written while block b is folded,
    // one barrier per block (the folds of consecutive blocks stay ordered)
    put(0, stage, lkey);
    fetch(0, kBfAhead);
    __syncthreads();   // acc cleared, block 0 staged
    for (int64_t b0 = 0; b0 < nblk; b0 += kBfAhead) {
#pragma unroll
      for (int j = 0; j < kBfAhead; ++j) {
        const int64_t b = b0 + j;
        if (b >= nblk) break;
        const int cur = (int)(b & 1);
        if (b + 1 < nblk) {
          const int jn = (j + 1) % kBfAhead;
          put(jn, stage + (cur ^ 1) * kBfRows, lkey + (cur ^ 1) * kBfRows);
          fetch(jn, b + 1 + kBfAhead);
        }
        fold(stage + cur * kBfRows, lkey + cur * kBfRows);
        __syncthreads();   // this block folded, the next one staged
      }
    }
    return;
  }
  for (int64_t b0 = 0; b0 < nblk; b0 += kBfAhead) {
#pragma unroll
    for (int j = 0; j < kBfAhead; ++j) {
      const int64_t b = b0 + j;
      if (b >= nblk) break;
      __syncthreads();   // acc cleared, or the previous block's runs done with stage and lkey
      put(j, stage, lkey);
      __syncthreads();
      fetch(j, b + kBfAhead);   // in flight while this block and the next ones are folded
      fold(stage, lkey);
    }
  }
  __syncthreads();
}

// Workgroup (column c, part p) owns buckets [m0, m1) of column c.
template <typename T, bool DB>
__global__ __launch_bounds__(kBfT) void k_bf_fold(int64_t d, int k, Cols<T> cols, int parts,
                                                  int slots, const uint32_t *__restrict__ keys,
                                                  T *__restrict__ Y, int64_t ldy) {
  constexpr int NB = DB ? 2 : 1;   // staging buffers
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *acc = reinterpret_cast<T *>(smem_raw);                           // slots
  T *stage = acc + slots;                                             // NB kBfRows
  uint32_t *lkey = reinterpret_cast<uint32_t *>(stage + NB * kBfRows);  // NB kBfRows
  const int tid = threadIdx.x;
  const int c = blockIdx.x / parts, part = blockIdx.x - (blockIdx.x / parts) * parts;
  const uint32_t m0 = (uint32_t)((int64_t)k * part / parts);
  const uint32_t m1 = (uint32_t)((int64_t)k * (part + 1) / parts);
  for (uint32_t i = tid; i < m1 - m0; i += kBfT) acc[i] = T(0);
  bf_fold_column<T, DB>(d, bf_col(cols, c), keys, m0, m1, acc, stage, lkey);
  for (uint32_t i = tid; i < m1 - m0; i += kBfT) Y[(m0 + i) + (int64_t)c * ldy] = acc[i];
}

// ------------------------------------------------------------------ batched

// Persistent over every problem's key blocks: problem p's block b sorted
// into keyarea + key_off (as k_bf_keys); bad rows recorded for the problem.
__global__ __launch_bounds__(kBfT) void k_batch_bf_keys(int count, const ms_problem *__restrict__ P,
                                                        const BatchEntry *__restrict__ E,
                                                        const BatchTotals *__restrict__ tot,
                                                        unsigned char *__restrict__ keyarea,
                                                        int *pstatus, int *status) {
  __shared__ __align__(16) uint32_t key[kBfRows];
  const int tid = threadIdx.x;
  const int64_t total = tot->bk_items;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = batch_find_m<&BatchEntry::bk_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    const int64_t r0 = (it - e.bk_start) * kBfRows;
    const int32_t *h = Q.h;
    const int8_t *s = Q.s;
    const bool vec = (((uintptr_t)h & 15) | ((uintptr_t)s & 3)) == 0;
    bool bad = false;
    uint32_t v[4];
    bf_make_keys(Q.d, Q.k, h, s, r0, vec, v, bad);
    if (bad) {
      record_status(&pstatus[p], MS_ERR_RANGE);
      record_status(status, MS_ERR_RANGE);
    }
    // the scratch is reused by the next item: the sort's first LDS phase
    // stores only each thread's own positions before its barrier
    sort4096_regs(v, key);
    uint32_t *out = reinterpret_cast<uint32_t *>(keyarea + e.key_off) + r0;
    *reinterpret_cast<uint4 *>(out + 4 * tid) = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// Persistent over fold items (problem, column, bucket part).  RES = 0:
// column c of [A | B] (data T) into the problem's Y (k x nc, T, ld k);
// RES = 1: column c of its residual r (FP64, d x nrhs, ld d) into Yr (FP64,
// k x nrhs, ld k).
template <typename T, int RES>
__global__ __launch_bounds__(kBfT) void k_batch_bf_fold(int count, const ms_problem *__restrict__ P,
                                                        const BatchEntry *__restrict__ E,
                                                        const BatchTotals *__restrict__ tot,
                                                        const unsigned char *__restrict__ keyarea,
                                                        const unsigned char *__restrict__ rarea,
                                                        unsigned char *__restrict__ out,
                                                        int slots) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *acc = reinterpret_cast<T *>(smem_raw);
  T *stage = acc + slots;
  uint32_t *lkey = reinterpret_cast<uint32_t *>(stage + kBfRows);
  const int tid = threadIdx.x;
  const int64_t total = RES ? tot->bfr_items : tot->bf_items;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = RES ? batch_find_m<&BatchEntry::bfr_start>(E, count, it)
                      : batch_find_m<&BatchEntry::bf_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    if (RES && !e.refine) continue;   // converged in an earlier step
    const int parts = RES ? e.rparts : e.parts;
    const int64_t local = it - (RES ? e.bfr_start : e.bf_start);
    const int c = (int)(local / parts), part = (int)(local - (local / parts) * parts);
    const uint32_t m0 = (uint32_t)(Q.k * part / parts);
    const uint32_t m1 = (uint32_t)(Q.k * (part + 1) / parts);
    const T *col;
    T *Yc;
    if (RES) {
      col = reinterpret_cast<const T *>(rarea + e.r_off) + (int64_t)c * Q.d;
      Yc = reinterpret_cast<T *>(out + e.yr_off) + (int64_t)c * Q.k;
    } else {
      col = c < Q.n ? static_cast<const T *>(Q.A) + (int64_t)c * Q.lda
                    : static_cast<const T *>(Q.B) + (int64_t)(c - Q.n) * Q.ldb;
      Yc = reinterpret_cast<T *>(out + e.y_off) + (int64_t)c * Q.k;
    }
    for (uint32_t i = tid; i < m1 - m0; i += kBfT) acc[i] = T(0);
    bf_fold_column<T>(Q.d, col, reinterpret_cast<const uint32_t *>(keyarea + e.key_off), m0, m1,
                      acc, stage, lkey);
    for (uint32_t i = tid; i < m1 - m0; i += kBfT) Yc[m0 + i] = acc[i];
    __syncthreads();   // acc is cleared by the next item
  }
}

struct BfShape {
  int parts = 0, slots = 0;
  size_t lds = 0;
};

BfShape bf_shape(int64_t k, int ncols, size_t elem, int bufs = 1) {
  BfShape s;
  if (k < 1 || k > kBfMaxK || ncols < 1) return s;
  const size_t fixed = (size_t)bufs * kBfRows * (elem + 4);
  const size_t avail = (size_t)dev_info().lds_per_block;
  if (avail <= fixed + 256 * elem) return s;
  const int64_t per = (int64_t)((avail - fixed) / elem);   // bucket sums one workgroup holds
  int parts = (int)((k + per - 1) / per);
  // spread a few columns over more workgroups (each part re-reads the column)
  const int want = std::max(1, std::min(8, 256 / std::max(1, ncols)));
  parts = std::max(parts, (int)std::min<int64_t>(want, k));
  if (parts > kBfMaxParts) return s;
  s.parts = parts;
  // a multiple of 4 slots keeps the staged keys 16-byte aligned (vector reads)
  s.slots = (int)(((k + parts - 1) / parts + 3) / 4 * 4);
  s.lds = (size_t)s.slots * elem + fixed;
  if (s.lds > avail) return BfShape{};
  return s;
}

}  // namespace

bool cs_blockfold_supported(int64_t d, int64_t k, int ncols, size_t elem) {
  return d >= 1 && d <= 0x7ffffffe && bf_shape(k, ncols, elem).parts > 0;
}

size_t cs_blockfold_key_bytes(int64_t d) {
  const int64_t nblk = (d + kBfRows - 1) / kBfRows;
  return align_up((size_t)nblk * kBfRows * 4);
}

hipError_t launch_bf_keys(int64_t d, int64_t k, const int32_t *h, const int8_t *s, uint32_t *keys,
                          int *status, hipStream_t st) {
  if (d < 1 || k < 1 || k > kBfMaxK) return hipErrorInvalidValue;
  const int64_t nblk = (d + kBfRows - 1) / kBfRows;
  if (k <= kBfCountMaxK) {
    const size_t lds = bf_count_lds(k);
    hipError_t e = allow_dynamic_lds((const void *)k_bf_keys_count, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bf_keys_count, dim3((unsigned)nblk), dim3(kBfT), lds, st, d, (int)k, h, s,
                       keys, status);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_bf_keys, dim3((unsigned)nblk), dim3(kBfT), 0, st, d, (int)k, h, s, keys,
                     status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bf_fold(int64_t d, int64_t k, const Cols<T> &c, const uint32_t *keys, T *Y,
                          int64_t ldy, hipStream_t st) {
  const BfShape sh = bf_shape(k, c.ncols, sizeof(T));
  if (!sh.parts) return hipErrorInvalidValue;
  // two staging buffers when they leave the same workgroup count
  const BfShape sh2 = bf_shape(k, c.ncols, sizeof(T), 2);
  const bool db = sh2.parts == sh.parts;
  const BfShape &u = db ? sh2 : sh;
  const void *fn = db ? (const void *)k_bf_fold<T, true> : (const void *)k_bf_fold<T, false>;
  hipError_t e = allow_dynamic_lds(fn, (int)u.lds);
  if (e != hipSuccess) return e;
  const int64_t grid = (int64_t)c.ncols * u.parts;
  if (db)
    hipLaunchKernelGGL((k_bf_fold<T, true>), dim3((unsigned)grid), dim3(kBfT), u.lds, st, d,
                       (int)k, c, u.parts, u.slots, keys, Y, ldy);
  else
    hipLaunchKernelGGL((k_bf_fold<T, false>), dim3((unsigned)grid), dim3(kBfT), u.lds, st, d,
                       (int)k, c, u.parts, u.slots, keys, Y, ldy);
  return hipGetLastError();
}
hipError_t launch_batch_bf_keys(int count, const ms_problem *P, const BatchEntry *E,
                                const BatchTotals *tot, unsigned char *keyarea, int *pstatus,
                                int *status, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_bf_keys, dim3((unsigned)grid), dim3(kBfT), 0, st, count, P, E, tot,
                     keyarea, pstatus, status);
  return hipGetLastError();
}

template <typename T, int RES>
hipError_t launch_batch_bf_fold(int count, const ms_problem *P, const BatchEntry *E,
                                const BatchTotals *tot, const unsigned char *keyarea,
                                const unsigned char *rarea, unsigned char *out, int grid,
                                hipStream_t st) {
  const int slots = (int)batch_bf_slots((int)sizeof(T));
  const size_t lds = (size_t)slots * sizeof(T) + (size_t)kBfRows * (sizeof(T) + 4);
  if (lds > (size_t)dev_info().lds_per_block) return hipErrorInvalidValue;
  const void *fn = (const void *)k_batch_bf_fold<T, RES>;
  hipError_t e = allow_dynamic_lds(fn, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch_bf_fold<T, RES>), dim3((unsigned)grid), dim3(kBfT), lds, st, count,
                     P, E, tot, keyarea, rarea, out, slots);
  return hipGetLastError();
}
template hipError_t launch_batch_bf_fold<float, 0>(int, const ms_problem *, const BatchEntry *,
                                                   const BatchTotals *, const unsigned char *,
                                                   const unsigned char *, unsigned char *, int,
                                                   hipStream_t);
template hipError_t launch_batch_bf_fold<double, 0>(int, const ms_problem *, const BatchEntry *,
                                                    const BatchTotals *, const unsigned char *,
                                                    const unsigned char *, unsigned char *, int,
                                                    hipStream_t);
template hipError_t launch_batch_bf_fold<double, 1>(int, const ms_problem *, const BatchEntry *,
                                                    const BatchTotals *, const unsigned char *,
                                                    const unsigned char *, unsigned char *, int,
                                                    hipStream_t);

template hipError_t launch_bf_fold<double>(int64_t, int64_t, const Cols<double> &,
                                           const uint32_t *, double *, int64_t, hipStream_t);
template hipError_t launch_bf_fold<float>(int64_t, int64_t, const Cols<float> &, const uint32_t *,
                                          float *, int64_t, hipStream_t);

}  // namespace ms
