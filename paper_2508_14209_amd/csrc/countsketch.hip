// countsketch.hip -- CountSketch Y = S [A | B] on gfx950 (Def. 3, Eq. (2),
// Alg. 2 of Higgins, Boman, Yamazaki, arXiv 2508.14209) and the sketch plan
// (bucket histogram, scan, stable counting sort) that its deterministic mode
// uses.
//
// A is column-major, so a column is a contiguous stream.  Three ways of
// forming the bucket sums of Eq. (2):
//   * atomic  -- Alg. 2 as written, one device-scope atomic add per element
//                (kept as the measured baseline);
//   * lds     -- each workgroup streams a row chunk of one column tile with
//                16-byte loads and accumulates bucket partial sums in LDS
//                (LDS atomics), then adds its partials to Y once;
//   * sorted  -- rows grouped by bucket by a stable counting sort, each
//                (bucket, column) folded sequentially in ascending row order
//                from +0.0: bit-identical to the sequential reading of Alg. 2.
#include <algorithm>
#include <type_traits>

#include "ms_internal.h"

namespace ms {

// ------------------------------------------------------------------ helpers

__global__ void k_zero_status(int *status) {
  if (threadIdx.x == 0) *status = MS_OK;
}

hipError_t launch_zero_status(int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, st, status);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill_zero(T *Y, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / rows;
    Y[(t - c * rows) + c * ld] = T(0);
  }
}

template <typename T>
hipError_t launch_fill_zero(T *Y, int64_t rows, int64_t cols, int64_t ld, hipStream_t st) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, st, Y, rows, cols, ld);
  return hipGetLastError();
}
template hipError_t launch_fill_zero<double>(double *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_fill_zero<float>(float *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_fill_zero<int32_t>(int32_t *, int64_t, int64_t, int64_t, hipStream_t);

// Start of a call: clear the status word and a buffer (the sketch that the
// atomic variants accumulate into, or the plan's bucket counts).
template <typename T>
__global__ void k_prologue(int *status, T *Y, int64_t rows, int64_t cols, int64_t ld) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = MS_OK;
  const int64_t total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / rows;
    Y[(t - c * rows) + c * ld] = T(0);
  }
}

template <typename T>
hipError_t launch_prologue(int *status, T *Y, int64_t rows, int64_t cols, int64_t ld,
                           hipStream_t st) {
  const int64_t total = std::max<int64_t>(0, rows * cols);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(k_prologue<T>, dim3((unsigned)blocks), dim3(256), 0, st, status, Y, rows, cols,
                     ld);
  return hipGetLastError();
}
template hipError_t launch_prologue<double>(int *, double *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_prologue<float>(int *, float *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t launch_prologue<int32_t>(int *, int32_t *, int64_t, int64_t, int64_t,
                                             hipStream_t);

// Validate (h, s) and pack them: code = h | (s == -1 ? sign bit : 0).  A row
// with h outside [0,k) or s not in {+1,-1} records MS_ERR_RANGE and is
// packed as bucket 0 so no later kernel leaves its bounds.
__global__ void k_pack_codes(int64_t d, int64_t k, const int32_t *__restrict__ h,
                             const int8_t *__restrict__ s, uint32_t *__restrict__ code,
                             int *status) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = h[i];
    const int8_t sg = s[i];
    const bool ok = b >= 0 && (int64_t)b < k && (sg == 1 || sg == -1);
    code[i] = ok ? ((uint32_t)b | (sg < 0 ? kSignBit : 0u)) : 0u;
    bad |= !ok;
  }
  if (bad) record_status(status, MS_ERR_RANGE);
}

hipError_t launch_pack_codes(int64_t d, int64_t k, const int32_t *h, const int8_t *s,
                             uint32_t *code, int *status, hipStream_t st) {
  if (d <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((d + 255) / 256, 8192);
  hipLaunchKernelGGL(k_pack_codes, dim3((unsigned)blocks), dim3(256), 0, st, d, k, h, s, code,
                     status);
  return hipGetLastError();
}

// ------------------------------------------------------------------ plan

// cnt[m] += 1 per row with h = m (integer atomics: the counts are exact and
// independent of order).
__global__ void k_hist(int64_t d, int64_t k, const int32_t *__restrict__ h,
                       int32_t *__restrict__ cnt, int *status) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = h[i];
    if (b >= 0 && (int64_t)b < k)
      atomicAdd(&cnt[b], 1);
    else
      bad = true;
  }
  if (bad) record_status(status, MS_ERR_RANGE);
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan of cnt into off (k+1 entries) by one workgroup of 1024
// threads, 4096 entries per pass with a running carry; also seeds the
// scatter cursors with the bucket offsets.
__global__ __launch_bounds__(1024) void k_scan(int64_t k, const int32_t *__restrict__ cnt,
                                               int32_t *__restrict__ off,
                                               int32_t *__restrict__ cursor) {
  __shared__ int32_t wave_tot[16];
  __shared__ int32_t carry_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < k; base += 4096) {
    int32_t v[4];
    int32_t local = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t idx = base + tid * 4 + q;
      v[q] = idx < k ? cnt[idx] : 0;
      local += v[q];
    }
    const int32_t incl = wave_incl_scan(local);
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    int32_t wave_off = 0;
    for (int w = 0; w < wave; ++w) wave_off += wave_tot[w];
    int32_t run = carry_s + wave_off + incl - local;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t idx = base + tid * 4 + q;
      if (idx < k) {
        off[idx] = run;
        cursor[idx] = run;
      }
      run += v[q];
    }
    __syncthreads();
    if (tid == 1023) carry_s = run;
    __syncthreads();
  }
  if (tid == 0) off[k] = carry_s;
}

// Scatter each row to a free slot of its bucket (order inside a bucket is
// arbitrary here and is fixed by the per-bucket sort that follows).
__global__ void k_scatter(int64_t d, int64_t k, const int32_t *__restrict__ h,
                          const int8_t *__restrict__ s, int32_t *__restrict__ cursor,
                          uint32_t *__restrict__ sperm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = h[i];
    if (b < 0 || (int64_t)b >= k) continue;
    const int32_t pos = atomicAdd(&cursor[b], 1);
    sperm[pos] = (uint32_t)i | ((s != nullptr && s[i] < 0) ? kSignBit : 0u);
  }
}

// Sort one bucket's entries by row index (bits 0..30) with a bitonic network
// in LDS.  Buckets of length <= CAP handled here; longer ones by the larger
// instantiation; lengths beyond MS_SORTED_MAX_SEGMENT are reported.
template <int CAP, int NTHREADS>
__global__ __launch_bounds__(NTHREADS) void k_segsort(int64_t k, int lo_exclusive,
                                                      const int32_t *__restrict__ off,
                                                      uint32_t *__restrict__ sperm,
                                                      int *status) {
  __shared__ uint32_t key[CAP];
  const int64_t b = blockIdx.x;
  if (b >= k) return;
  const int32_t o0 = off[b];
  const int len = off[b + 1] - o0;
  if (len <= lo_exclusive || len < 2) return;
  if (len > CAP) {
    if (CAP >= MS_SORTED_MAX_SEGMENT && threadIdx.x == 0) record_status(status, MS_ERR_UNSUPPORTED);
    return;
  }
  int P = 2;
  while (P < len) P <<= 1;
  for (int t = threadIdx.x; t < P; t += NTHREADS) key[t] = t < len ? sperm[o0 + t] : 0xffffffffu;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (P >> 1); t += NTHREADS) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint32_t a = key[lo], c = key[hi];
        if (((a & kIdxMask) > (c & kIdxMask)) == up) {
          key[lo] = c;
          key[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < len; t += NTHREADS) sperm[o0 + t] = key[t];
}

hipError_t launch_plan(int64_t d, int64_t k, const int32_t *h, const int8_t *s, int32_t *cnt,
                       int32_t *off, int32_t *cursor, uint32_t *sperm, int *status,
                       hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((d + 255) / 256, 8192));
  if (d > 0) hipLaunchKernelGGL(k_hist, dim3((unsigned)blocks), dim3(256), 0, st, d, k, h, cnt, status);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, k, cnt, off, cursor);
  if (d > 0)
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, st, d, k, h, s, cursor,
                       sperm);
  // buckets of length 2..1024, then 1025..MS_SORTED_MAX_SEGMENT
  hipLaunchKernelGGL((k_segsort<1024, 256>), dim3((unsigned)k), dim3(256), 0, st, k, 0, off,
                     sperm, status);
  hipLaunchKernelGGL((k_segsort<MS_SORTED_MAX_SEGMENT, 1024>), dim3((unsigned)k), dim3(1024), 0,
                     st, k, 1024, off, sperm, status);
  return hipGetLastError();
}

__global__ void k_strip_sign(int64_t d, const uint32_t *__restrict__ sperm,
                             int32_t *__restrict__ perm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x)
    perm[i] = (int32_t)(sperm[i] & kIdxMask);
}

hipError_t launch_strip_sign(int64_t d, const uint32_t *sperm, int32_t *perm, hipStream_t st) {
  if (d <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((d + 255) / 256, 8192);
  hipLaunchKernelGGL(k_strip_sign, dim3((unsigned)blocks), dim3(256), 0, st, d, sperm, perm);
  return hipGetLastError();
}

// ------------------------------------------------------------------ column access

template <typename T>
__device__ __forceinline__ const T *col_ptr(const Cols<T> &c, int j) {
  return j < c.n_a ? c.A + (int64_t)j * c.lda : c.B + (int64_t)(j - c.n_a) * c.ldb;
}

// ------------------------------------------------------------------ atomic (Alg. 2)

// One thread per (row, column): Y[h[i], c] += +-A[i, c] with a device-scope
// floating-point atomic add.  Y must be zero on entry.
template <typename T>
__global__ __launch_bounds__(256) void k_cs_atomic(int64_t d, int64_t k, Cols<T> cols,
                                                   const uint32_t *__restrict__ code,
                                                   T *__restrict__ Y, int64_t ldy, int *status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= d) return;
  const uint32_t cd = code[i];
  const int64_t b = (int64_t)(cd & kIdxMask);
  if (b >= k) {
    record_status(status, MS_ERR_RANGE);
    return;
  }
  const T a = col_ptr(cols, c)[i];
  unsafeAtomicAdd(&Y[b + (int64_t)c * ldy], apply_sign(a, cd));
}

template <typename T>
hipError_t launch_cs_atomic(int64_t d, int64_t k, const Cols<T> &c, const uint32_t *code, T *Y,
                            int64_t ldy, bool zero_first, int *status, hipStream_t st) {
  hipError_t e = zero_first ? launch_fill_zero<T>(Y, k, c.ncols, ldy, st) : hipSuccess;
  if (e != hipSuccess || d <= 0 || c.ncols <= 0) return e;
  for (int c0 = 0; c0 < c.ncols; c0 += 65535) {
    Cols<T> sub = c;
    const int nc = std::min(65535, c.ncols - c0);
    // shift the column window: columns c0.. of [A | B]
    if (c0 < c.n_a) {
      sub.A = c.A + (int64_t)c0 * c.lda;
      sub.n_a = c.n_a - c0;
    } else {
      sub.A = nullptr;
      sub.B = c.B + (int64_t)(c0 - c.n_a) * c.ldb;
      sub.n_a = 0;
    }
    sub.ncols = nc;
    hipLaunchKernelGGL(k_cs_atomic<T>, dim3((unsigned)((d + 255) / 256), nc), dim3(256), 0, st, d,
                       k, sub, code, Y + (int64_t)c0 * ldy, ldy, status);
  }
  return hipGetLastError();
}
template hipError_t launch_cs_atomic<double>(int64_t, int64_t, const Cols<double> &,
                                             const uint32_t *, double *, int64_t, bool, int *,
                                             hipStream_t);
template hipError_t launch_cs_atomic<float>(int64_t, int64_t, const Cols<float> &,
                                            const uint32_t *, float *, int64_t, bool, int *,
                                            hipStream_t);

// ------------------------------------------------------------------ LDS-binned

// 16-byte vector types for the streaming loads of the data columns, aligned
// only to their element: a column of leading dimension d starts at any
// element, and a dword-aligned multi-dword global load is legal on CDNA, so
// every d takes the vector path (a wave's 1 KB then spans one more cache
// line when the column start is not 16-byte aligned).
template <typename T>
struct Vec16;
typedef double dvec2 __attribute__((ext_vector_type(2), aligned(8)));
typedef float fvec4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t uvec2 __attribute__((ext_vector_type(2)));
typedef uint32_t uvec4 __attribute__((ext_vector_type(4)));
template <>
struct Vec16<double> {
  using type = dvec2;
  static constexpr int N = 2;
  using code_t = uvec2;
};
template <>
struct Vec16<float> {
  using type = fvec4;
  static constexpr int N = 4;
  using code_t = uvec4;
};

template <typename T>
__device__ __forceinline__ T lane_of(const typename Vec16<T>::type &v, int q) {
  return v[q];
}
template <typename CV>
__device__ __forceinline__ uint32_t code_of(const CV &v, int q) {
  return v[q];
}

// Where a row's bucket and sign come from (the SRC template argument).
constexpr int kSrcHS = 0;    // stored h and s, checked per row
constexpr int kSrcCode = 1;  // packed 4-byte words (ms_pack_sketch)
constexpr int kSrcHash = 2;  // generated from (key, row): the hash-generated sketch

// The hash-generated sketch's word of row i: u = SplitMix64's (i+1)-th output
// from state key (Steele, Lea and Flood, OOPSLA 2014: state += 0x9E3779B97F4A7C15,
// output = the state through its finaliser); bucket = the top 32 bits of u
// times k, shifted down 32 (multiply-shift, < k); sign bit = bit 0 of u.
__device__ __forceinline__ uint32_t hash_word(uint64_t key, int64_t i, int64_t k) {
  uint64_t z = key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  const uint32_t b = (uint32_t)(((z >> 32) * (uint64_t)k) >> 32);
  return b | ((uint32_t)z << 31);
}

// The bucket/sign word of row i: a packed code (kSrcCode), a generated word
// (kSrcHash, always valid), or built from h and s (kSrcHS), in which case a
// row with h outside [0,k) or s not +-1 yields an invalid word (bucket field
// 0x7fffffff, never inside a tile) and sets bad.
template <int SRC>
__device__ __forceinline__ uint32_t row_word(const uint32_t *__restrict__ code,
                                             const int32_t *__restrict__ h,
                                             const int8_t *__restrict__ s, int64_t i, int64_t k,
                                             bool &bad, uint64_t key = 0) {
  if (SRC == kSrcHash) return hash_word(key, i, k);
  if (SRC == kSrcCode) {
    const uint32_t e = gload(code + i);
    bad |= (int64_t)(e & kIdxMask) >= k;
    return e;
  }
  const int32_t b = gload(h + i);
  const int8_t sg = gload(s + i);
  // bitwise, not short-circuit: no branch per row (k < 2^31 is checked by
  // every caller, so one unsigned compare covers 0 <= b < k)
  const bool ok = ((uint32_t)b < (uint32_t)k) & ((sg == 1) | (sg == -1));
  bad |= !ok;
  return ok ? ((uint32_t)b | (sg < 0 ? kSignBit : 0u)) : 0xffffffffu;
}

typedef int32_t ivec2 __attribute__((ext_vector_type(2)));
typedef int32_t ivec4 __attribute__((ext_vector_type(4)));
typedef int8_t cvec2 __attribute__((ext_vector_type(2)));
typedef int8_t cvec4 __attribute__((ext_vector_type(4)));
template <int W>
struct HsVec;
template <>
struct HsVec<2> {
  using hv = ivec2;
  using sv = cvec2;
};
template <>
struct HsVec<4> {
  using hv = ivec4;
  using sv = cvec4;
};

// W consecutive words starting at row i (i a multiple of W; 16/8/4/2-byte
// aligned loads).
template <int SRC, int W>
__device__ __forceinline__ void row_words(const uint32_t *__restrict__ code,
                                          const int32_t *__restrict__ h,
                                          const int8_t *__restrict__ s, int64_t i, int64_t k,
                                          uint32_t (&e)[W], bool &bad, uint64_t key = 0) {
  if (SRC == kSrcHash) {
#pragma unroll
    for (int q = 0; q < W; ++q) e[q] = hash_word(key, i + q, k);
  } else if (SRC == kSrcCode) {
    using CV = typename Vec16<typename std::conditional<W == 2, double, float>::type>::code_t;
    const CV v = gload(reinterpret_cast<const CV *>(code + i));
#pragma unroll
    for (int q = 0; q < W; ++q) {
      e[q] = v[q];
      bad |= (int64_t)(e[q] & kIdxMask) >= k;
    }
  } else {
    const typename HsVec<W>::hv hv = gload(reinterpret_cast<const typename HsVec<W>::hv *>(h + i));
    const typename HsVec<W>::sv sv = gload(reinterpret_cast<const typename HsVec<W>::sv *>(s + i));
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const int32_t b = hv[q];
      const int8_t sg = sv[q];
      const bool ok = ((uint32_t)b < (uint32_t)k) & ((sg == 1) | (sg == -1));
      bad |= !ok;
      e[q] = ok ? ((uint32_t)b | (sg < 0 ? kSignBit : 0u)) : 0xffffffffu;
    }
  }
}

// Workgroup (chunk, column tile, bucket tile): rows [r0, r1) of NT columns
// starting at c0, buckets [b0, b0 + kt).  Partial sums live in LDS as
// acc[b + j*kt]; rows whose bucket is outside the tile are skipped (only
// when the buckets of a column do not fit in LDS at once).  Y += the
// partials, one atomic add per non-zero partial.
template <typename T, int NT, bool VEC, int SRC>
__global__ __launch_bounds__(1024) void k_cs_lds(int64_t d, Cols<T> cols,
                                                 const uint32_t *__restrict__ code,
                                                 const int32_t *__restrict__ h,
                                                 const int8_t *__restrict__ s, int64_t k,
                                                 int64_t ktile, int64_t rows_per_chunk,
                                                 T *__restrict__ Y, int64_t ldy, int *status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);
  const int64_t b0 = (int64_t)blockIdx.z * ktile;
  const uint32_t kt = (uint32_t)min(ktile, k - b0);
  const int c0 = blockIdx.y * NT;
  const int nc = min(NT, cols.ncols - c0);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = min(d, r0 + rows_per_chunk);
  bool bad = false;

  for (uint32_t t = threadIdx.x; t < kt * NT; t += blockDim.x) acc[t] = 0.0;
  const T *cp[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) cp[j] = col_ptr(cols, min(c0 + j, cols.ncols - 1));
  __syncthreads();

  if (VEC) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::N;
    const int64_t step = (int64_t)blockDim.x * W;
    int64_t i = r0 + (int64_t)threadIdx.x * W;
    // two vectors in flight per thread per iteration
    for (; i + step + W <= r1; i += 2 * step) {
      uint32_t e0[W], e1[W];
      row_words<SRC, W>(code, h, s, i, k, e0, bad, cols.key);
      row_words<SRC, W>(code, h, s, i + step, k, e1, bad, cols.key);
      V a0[NT], a1[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        a0[j] = gload_nt(reinterpret_cast<const V *>(cp[j] + i));
        a1[j] = gload_nt(reinterpret_cast<const V *>(cp[j] + i + step));
      }
#pragma unroll
      for (int q = 0; q < W; ++q) {
        const uint32_t l0 = (e0[q] & kIdxMask) - (uint32_t)b0;
        const uint32_t l1 = (e1[q] & kIdxMask) - (uint32_t)b0;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          if (j < nc) {
            if (l0 < kt) atomicAdd(&acc[l0 + j * kt], (double)apply_sign(lane_of<T>(a0[j], q), e0[q]));
            if (l1 < kt) atomicAdd(&acc[l1 + j * kt], (double)apply_sign(lane_of<T>(a1[j], q), e1[q]));
          }
        }
      }
    }
    for (; i < r1; i += step) {
      if (i + W <= r1) {
        uint32_t e0[W];
        row_words<SRC, W>(code, h, s, i, k, e0, bad, cols.key);
        V a0[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) a0[j] = gload(reinterpret_cast<const V *>(cp[j] + i));
#pragma unroll
        for (int q = 0; q < W; ++q) {
          const uint32_t l0 = (e0[q] & kIdxMask) - (uint32_t)b0;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            if (j < nc && l0 < kt) atomicAdd(&acc[l0 + j * kt], (double)apply_sign(lane_of<T>(a0[j], q), e0[q]));
        }
      } else {
        for (int64_t r = i; r < r1; ++r) {
          const uint32_t e0 = row_word<SRC>(code, h, s, r, k, bad, cols.key);
          const uint32_t l0 = (e0 & kIdxMask) - (uint32_t)b0;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            if (j < nc && l0 < kt) atomicAdd(&acc[l0 + j * kt], (double)apply_sign(gload(cp[j] + r), e0));
        }
      }
    }
  } else {
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const uint32_t e0 = row_word<SRC>(code, h, s, r, k, bad, cols.key);
      const uint32_t l0 = (e0 & kIdxMask) - (uint32_t)b0;
#pragma unroll
      for (int j = 0; j < NT; ++j)
        if (j < nc && l0 < kt) atomicAdd(&acc[l0 + j * kt], (double)apply_sign(gload(cp[j] + r), e0));
    }
  }
  if (bad) record_status(status, MS_ERR_RANGE);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < kt * (uint32_t)nc; t += blockDim.x) {
    const uint32_t j = t / kt, b = t - j * kt;
    const double v = acc[t];
    if (v != 0.0) unsafeAtomicAdd(&Y[(b0 + b) + (int64_t)(c0 + j) * ldy], (T)v);
  }
}

// ------------------------------------------------------------------ persistent, XCD-aware

// Rows [r0, r1) of column tile ct (NT columns from c0) and bucket tile
// [b0, b0 + kt): accumulate into LDS (zero on entry), then add the non-zero
// partials to Y (PST: store every partial, zeros included, into a buffer the
// workgroup owns) and leave LDS zero again.  UNR vectors in flight per thread.
template <typename T, int NT, bool VEC, int SRC, int UNR, bool NTL, bool PST = false>
__device__ __forceinline__ void cs_segment(double *acc, const Cols<T> &cols, int c0, int nc,
                                           const uint32_t *__restrict__ code,
                                           const int32_t *__restrict__ h,
                                           const int8_t *__restrict__ s, int64_t k, int64_t b0,
                                           uint32_t kt, int64_t r0, int64_t r1,
                                           T *__restrict__ Y, int64_t ldy, bool &bad) {
  const T *cp[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) cp[j] = col_ptr(cols, min(c0 + j, cols.ncols - 1));
  auto scalar_row = [&](int64_t r) {
    const uint32_t e0 = row_word<SRC>(code, h, s, r, k, bad, cols.key);
    const uint32_t l0 = (e0 & kIdxMask) - (uint32_t)b0;
#pragma unroll
    for (int j = 0; j < NT; ++j)
      if (j < nc && l0 < kt) atomicAdd(&acc[l0 + j * kt], (double)apply_sign(gload(cp[j] + r), e0));
  };
  if (VEC) {
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::N;
    // head rows up to the first multiple of W
    const int64_t ra = min(r1, (r0 + W - 1) / W * W);
    for (int64_t r = r0 + threadIdx.x; r < ra; r += blockDim.x) scalar_row(r);
    const int64_t step = (int64_t)blockDim.x * W;
    int64_t i = ra + (int64_t)threadIdx.x * W;
    for (; i + (UNR - 1) * step + W <= r1; i += UNR * step) {
      uint32_t e[UNR][W];
      V a[UNR][NT];
#pragma unroll
      for (int u = 0; u < UNR; ++u) row_words<SRC, W>(code, h, s, i + u * step, k, e[u], bad, cols.key);
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int j = 0; j < NT; ++j)
          a[u][j] = NTL ? gload_nt(reinterpret_cast<const V *>(cp[j] + i + u * step))
                        : gload(reinterpret_cast<const V *>(cp[j] + i + u * step));
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int q = 0; q < W; ++q) {
          const uint32_t l = (e[u][q] & kIdxMask) - (uint32_t)b0;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            if (j < nc && l < kt) atomicAdd(&acc[l + j * kt], (double)apply_sign(lane_of<T>(a[u][j], q), e[u][q]));
        }
    }
    for (; i < r1; i += step) {
      if (i + W <= r1) {
        uint32_t e0[W];
        row_words<SRC, W>(code, h, s, i, k, e0, bad, cols.key);
        V a0[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) a0[j] = gload(reinterpret_cast<const V *>(cp[j] + i));
#pragma unroll
        for (int q = 0; q < W; ++q) {
          const uint32_t l0 = (e0[q] & kIdxMask) - (uint32_t)b0;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            if (j < nc && l0 < kt) atomicAdd(&acc[l0 + j * kt], (double)apply_sign(lane_of<T>(a0[j], q), e0[q]));
        }
      } else {
        for (int64_t r = i; r < r1; ++r) scalar_row(r);
      }
    }
  } else {
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) scalar_row(r);
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < kt * (uint32_t)nc; t += blockDim.x) {
    const uint32_t j = t / kt, b = t - j * kt;
    const double v = acc[t];
    acc[t] = 0.0;
    if (PST)
      Y[(b0 + b) + (int64_t)(c0 + j) * ldy] = (T)v;
    else if (v != 0.0)
      unsafeAtomicAdd(&Y[(b0 + b) + (int64_t)(c0 + j) * ldy], (T)v);
  }
  __syncthreads();
}

// Persistent grid of xcds * spx workgroups.  Workgroups are dispatched to the
// accelerator dies round-robin by id, so workgroup g runs on die g % xcds;
// die x owns rows [x*rpx, (x+1)*rpx), so the codes of those rows are shared
// in its L2.  On a die, slot s takes bucket tile s % nbt and an equal,
// contiguous share of the (column tile, row) space of its rows, so the bucket
// tiles of a column are streamed by workgroups of the same die at the same
// time, and each workgroup flushes LDS only when its share crosses a column
// tile.  PART: the die's groups split its column tiles instead (whole tiles,
// all of the die's rows), so each (column, bucket) of a die has one owner,
// which stores its partial sum into the die's slice of a partial buffer (Y,
// ld k, slices of k x ncols) with plain stores; k_cs_part_reduce adds the
// slices to the output.
template <typename T, int NT, bool VEC, int SRC, int UNR, bool NTL, bool PART>
__global__ __launch_bounds__(1024) void k_cs_lds_xcd(int64_t d, Cols<T> cols,
                                                     const uint32_t *__restrict__ code,
                                                     const int32_t *__restrict__ h,
                                                     const int8_t *__restrict__ s, int64_t k,
                                                     int64_t ktile, int nct, int nbt, int xcds,
                                                     int spx, int64_t rpx, T *__restrict__ Y,
                                                     int64_t ldy, int *status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);
  const int g = blockIdx.x;
  const int x = g % xcds, slot = g / xcds;
  const int subs = spx / nbt;
  if (slot >= subs * nbt) return;
  const int bt = slot % nbt, sub = slot / nbt;
  const int64_t R0 = (int64_t)x * rpx, R1 = min(d, R0 + rpx);
  if (R0 >= R1) return;
  const int64_t len = R1 - R0;
  const int64_t b0 = (int64_t)bt * ktile;
  const uint32_t kt = (uint32_t)min(ktile, k - b0);
  for (uint32_t t = threadIdx.x; t < kt * NT; t += blockDim.x) acc[t] = 0.0;
  __syncthreads();
  bool bad = false;
  if (PART) {
    const int ct0 = (int)((int64_t)nct * sub / subs), ct1 = (int)((int64_t)nct * (sub + 1) / subs);
    T *Px = Y + (int64_t)x * k * cols.ncols;
    for (int ct = ct0; ct < ct1; ++ct) {
      const int c0 = ct * NT;
      const int nc = min(NT, cols.ncols - c0);
      cs_segment<T, NT, VEC, SRC, UNR, NTL, true>(acc, cols, c0, nc, code, h, s, k, b0, kt, R0,
                                                    R1, Px, k, bad);
    }
    if (bad) record_status(status, MS_ERR_RANGE);
    return;
  }
  const int64_t total = (int64_t)nct * len;
  int64_t u0 = (total * sub / subs) & ~(int64_t)255;
  const int64_t u1 = sub + 1 == subs ? total : ((total * (sub + 1) / subs) & ~(int64_t)255);
  while (u0 < u1) {
    const int ct = (int)(u0 / len);
    const int64_t rlo = u0 - (int64_t)ct * len;
    const int64_t rhi = min(len, rlo + (u1 - u0));
    const int c0 = ct * NT;
    const int nc = min(NT, cols.ncols - c0);
    cs_segment<T, NT, VEC, SRC, UNR, NTL>(acc, cols, c0, nc, code, h, s, k, b0, kt, R0 + rlo,
                                            R0 + rhi, Y, ldy, bad);
    u0 += rhi - rlo;
  }
  if (bad) record_status(status, MS_ERR_RANGE);
}

// Y += the sum over dies (in die order, in FP64) of the per-die partial
// slices written by the PART schedule (slice x: k x ncols, ld k).
template <typename T>
__global__ void k_cs_part_reduce(int64_t k, int ncols, int ndies, const T *__restrict__ part,
                                 T *__restrict__ Y, int64_t ldy) {
  const int64_t total = k * ncols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / k, b = t - c * k;
    double s = 0.0;
    for (int x = 0; x < ndies; ++x) s += (double)part[t + (int64_t)x * total];
    T *y = Y + b + c * ldy;
    *y = (T)((double)*y + s);
  }
}

// Bytes of the per-die partial buffer when the PART schedule pays: the
// bucket range needs several LDS tiles (one column per tile), the atomic
// flushes of the die-row schedule (every bucket of every column once per
// die, 8 k per column) would exceed 1/16 of the data, and the columns split
// over a die's groups to within 25%.  0 otherwise.  Assumes 8 dies of 32
// compute units and 128 KB of LDS per workgroup (FP64 slots); the launch
// checks the device matches.
size_t cs_part_bytes(int64_t d, int64_t k, int64_t ncols, int64_t wd) {
  const int64_t ktile = (128 * 1024) / 8;
  if (k <= ktile || ncols < 1 || d < 1) return 0;
  const int64_t nbt = (k + ktile - 1) / ktile;
  const int64_t subs = 32 / nbt;
  if (subs < 1 || 128 * k < d) return 0;
  const int64_t per = (ncols + subs - 1) / subs;
  if (ncols < subs || per * subs * 4 > ncols * 5) return 0;
  return (size_t)(8 * k * ncols * wd);
}

// ------------------------------------------------------------------ batched

// Persistent workgroups over the CountSketch items of all problems: item =
// (problem, row segment, column tile, bucket tile).  h and s are read and
// validated in the kernel; a problem's Y must be zero on entry.  RES: the
// CountSketch of the FP64 residual columns (refinement) instead of [A | B].
template <typename T, bool RES>
__global__ __launch_bounds__(1024) void k_batch_cs(int count, const ms_problem *__restrict__ P,
                                                   const BatchEntry *__restrict__ E,
                                                   const BatchTotals *__restrict__ tot,
                                                   const unsigned char *__restrict__ codearea,
                                                   const unsigned char *__restrict__ rarea,
                                                   unsigned char *__restrict__ yarea,
                                                   int *__restrict__ pstatus, int *status,
                                                   int dies) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);
  for (int t = threadIdx.x; t < kBatchLdsSlots; t += blockDim.x) acc[t] = 0.0;
  __syncthreads();
  const int64_t total = RES ? tot->rcs_items : tot->cs_items;
  const DieOrder ord(dies);
  for (int64_t rr = 0;; ++rr) {
    const int64_t it = ord.item(rr);
    if (it >= total) break;
    const int p = RES ? batch_find_m<&BatchEntry::rcs_start>(E, count, it)
                      : batch_find_m<&BatchEntry::cs_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    if (RES && !e.refine) continue;   // converged in an earlier step
    const int nbt = RES ? e.rnbt : e.nbt, nt = RES ? e.rnt : e.nt;
    const int64_t ktile = RES ? e.rktile : e.ktile;
    // the column tiles and bucket tiles of a row segment are consecutive
    // items, so h and s of the segment are read from each die's L2 once
    // rather than once per column tile
    const int ntl = RES ? e.rntiles : e.ntiles;
    int64_t local = it - (RES ? e.rcs_start : e.cs_start);
    const int bt = (int)(local % nbt);
    local /= nbt;
    const int tile = (int)(local % ntl);
    const int seg = (int)(local / ntl);
    const int64_t r0 = (int64_t)seg * e.rows, r1 = min(Q.d, r0 + e.rows);
    const int64_t b0 = (int64_t)bt * ktile;
    const uint32_t kt = (uint32_t)min(ktile, Q.k - b0);
    Cols<T> cols;
    T *Y;
    // the packed words of the problem's rows (256-byte aligned: the vector
    // path), or, for problems swept only a few times (and in a replay with
    // more rows than the capacity), h and s read and checked by every item
    const bool packed = e.code_off >= 0;
    const bool vec = ((uintptr_t)Q.h & 15) == 0 &&
                     ((uintptr_t)Q.s & (uintptr_t)(16 / sizeof(T) - 1)) == 0;
    const uint32_t *code =
        packed ? reinterpret_cast<const uint32_t *>(codearea + e.code_off) : nullptr;
    if (RES) {
      const T *r = reinterpret_cast<const T *>(rarea + e.r_off);
      cols = Cols<T>{r, Q.d, nullptr, 0, (int)Q.nrhs, (int)Q.nrhs};
      Y = reinterpret_cast<T *>(yarea + e.yr_off);
    } else {
      cols = Cols<T>{static_cast<const T *>(Q.A), Q.lda, static_cast<const T *>(Q.B), Q.ldb,
                     (int)Q.n, e.nc};
      Y = reinterpret_cast<T *>(yarea + e.y_off);
    }
    const int c0 = tile * nt;
    const int ncur = min(nt, cols.ncols - c0);
    bool bad = false;
    // the tile width is a template argument, so narrow tiles issue no
    // loads for columns they do not have
#define MS_BCS_W(NT_, UNR_, NTL_, PST_)                                                      \
  if (packed)                                                                                      \
    cs_segment<T, NT_, true, true, UNR_, NTL_, PST_>(acc, cols, c0, ncur, code, nullptr, nullptr,  \
                                                     Q.k, b0, kt, r0, r1, Y, Q.k, bad);            \
  else if (vec)                                                                                    \
    cs_segment<T, NT_, true, false, UNR_, NTL_, PST_>(acc, cols, c0, ncur, nullptr, Q.h, Q.s, Q.k, \
                                                      b0, kt, r0, r1, Y, Q.k, bad);                \
  else                                                                                             \
    cs_segment<T, NT_, false, false, UNR_, false, PST_>(acc, cols, c0, ncur, nullptr, Q.h, Q.s,    \
                                                        Q.k, b0, kt, r0, r1, Y, Q.k, bad);
    // with one bucket tile each column value is read once: nontemporal loads
    // keep it from evicting the codes of the segment, which the other column
    // tiles read from L2.  With one row segment the item is the only
    // writer of its tile of the output: plain stores, and the output needs
    // no clearing beforehand.
#define MS_BCS_V(NT_, UNR_, NTL_)         \
  if (e.nsegs == 1) {                     \
    MS_BCS_W(NT_, UNR_, NTL_, true)       \
  } else {                                \
    MS_BCS_W(NT_, UNR_, NTL_, false)      \
  }
#define MS_BCS(NT_, UNR_)            \
  if (nbt == 1) {                    \
    MS_BCS_V(NT_, UNR_, true)        \
  } else {                           \
    MS_BCS_V(NT_, UNR_, false)       \
  }
    if (nt >= 4) {
      MS_BCS(4, 2)
    } else if (nt == 2) {
      MS_BCS(2, 4)
    } else {
      MS_BCS(1, 4)
    }
#undef MS_BCS
#undef MS_BCS_V
#undef MS_BCS_W
    if (bad) {
      record_status(&pstatus[p], MS_ERR_RANGE);
      record_status(status, MS_ERR_RANGE);
    }
  }
}

// The packed words of the rows of every problem that packs them (grid x
// over rows, four per thread with 16-byte loads of h when aligned; y over
// problems).
__global__ void k_batch_pack(int count, const ms_problem *__restrict__ P,
                             const BatchEntry *__restrict__ E, unsigned char *__restrict__ codearea,
                             int *__restrict__ pstatus, int *status) {
  for (int p = blockIdx.y; p < count; p += gridDim.y) {
    const BatchEntry &e = E[p];
    if (!e.valid || e.code_off < 0) continue;
    const ms_problem &Q = P[p];
    uint32_t *code = reinterpret_cast<uint32_t *>(codearea + e.code_off);
    const bool vec = ((uintptr_t)Q.h & 15) == 0 && ((uintptr_t)Q.s & 3) == 0;
    bool bad = false;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < Q.d;
         i += (int64_t)gridDim.x * blockDim.x * 4) {
      if (vec && i + 4 <= Q.d) {
        uint32_t w[4];
        row_words<false, 4>(nullptr, Q.h, Q.s, i, Q.k, w, bad);
        *reinterpret_cast<uvec4 *>(code + i) = uvec4{w[0], w[1], w[2], w[3]};
      } else {
        for (int64_t r = i; r < min(Q.d, i + 4); ++r) code[r] = row_word<false>(nullptr, Q.h, Q.s, r, Q.k, bad);
      }
    }
    if (bad) {
      record_status(&pstatus[p], MS_ERR_RANGE);
      record_status(status, MS_ERR_RANGE);
    }
  }
}

hipError_t launch_batch_pack(int count, const ms_problem *P, const BatchEntry *E,
                             unsigned char *codearea, int *pstatus, int *status, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_pack, dim3(128, (unsigned)std::min(count, 1024)), dim3(256), 0, st,
                     count, P, E, codearea, pstatus, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_cs(int count, const ms_problem *P, const BatchEntry *E,
                           const BatchTotals *tot, const unsigned char *codearea,
                           unsigned char *yarea, int *pstatus, int *status, int grid,
                           hipStream_t st) {
  const size_t lds = (size_t)kBatchLdsSlots * sizeof(double);
  hipError_t e = allow_dynamic_lds((const void *)k_batch_cs<T, false>, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch_cs<T, false>), dim3(grid), dim3(1024), lds, st, count, P, E, tot,
                     codearea, (const unsigned char *)nullptr, yarea, pstatus, status,
                     grid_dies(grid, dev_info().xcds));
  return hipGetLastError();
}
template hipError_t launch_batch_cs<double>(int, const ms_problem *, const BatchEntry *,
                                            const BatchTotals *, const unsigned char *,
                                            unsigned char *, int *, int *, int, hipStream_t);
template hipError_t launch_batch_cs<float>(int, const ms_problem *, const BatchEntry *,
                                           const BatchTotals *, const unsigned char *,
                                           unsigned char *, int *, int *, int, hipStream_t);

hipError_t launch_batch_cs_res(int count, const ms_problem *P, const BatchEntry *E,
                               const BatchTotals *tot, const unsigned char *codearea,
                               const unsigned char *rarea, unsigned char *yrarea, int *pstatus,
                               int *status, int grid, hipStream_t st) {
  const size_t lds = (size_t)kBatchLdsSlots * sizeof(double);
  hipError_t e = allow_dynamic_lds((const void *)k_batch_cs<double, true>, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch_cs<double, true>), dim3(grid), dim3(1024), lds, st, count, P, E,
                     tot, codearea, rarea, yrarea, pstatus, status,
                     grid_dies(grid, dev_info().xcds));
  return hipGetLastError();
}

template <typename T, int NT, bool VEC, int SRC, int UNR, bool NTL, bool PART>
static hipError_t launch_cs_xcd_k(int grid, size_t lds, hipStream_t st, int64_t d,
                                  const Cols<T> &c, const uint32_t *code, const int32_t *h,
                                  const int8_t *s, int64_t k, int64_t ktile, int nct, int nbt,
                                  int xcds, int spx, int64_t rpx, T *Y, int64_t ldy, int *status) {
  const void *fn = (const void *)k_cs_lds_xcd<T, NT, VEC, SRC, UNR, NTL, PART>;
  hipError_t e = allow_dynamic_lds(fn, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_cs_lds_xcd<T, NT, VEC, SRC, UNR, NTL, PART>), dim3(grid), dim3(1024),
                     lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, Y, ldy,
                     status);
  return hipGetLastError();
}

// part (may be null): per-die partial buffer of xcds * k * ncols elements;
// when given (one column per tile only), the PART schedule stores into it and
// k_cs_part_reduce adds it to Y.
template <typename T, int NT, int SRC>
static hipError_t launch_cs_xcd_v(bool vec, int grid, size_t lds, hipStream_t st, int64_t d,
                                  const Cols<T> &c, const uint32_t *code, const int32_t *h,
                                  const int8_t *s, int64_t k, int64_t ktile, int nct, int nbt,
                                  int xcds, int spx, int64_t rpx, T *Y, int64_t ldy, T *part,
                                  int *status) {
  // vectors in flight per thread: fewer for wider column tiles (registers)
  constexpr int UNR = NT >= 8 ? 1 : NT >= 4 ? 2 : 4;
  if constexpr (NT == 1) {
  if (part && nbt > 1) {
    hipError_t e =
        vec ? launch_cs_xcd_k<T, NT, true, SRC, UNR, false, true>(
                  grid, lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, part, k,
                  status)
            : launch_cs_xcd_k<T, NT, false, SRC, UNR, false, true>(
                  grid, lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, part, k,
                  status);
    if (e != hipSuccess) return e;
    const int ndies = (int)std::min<int64_t>(xcds, (d + rpx - 1) / rpx);
    const int64_t total = k * c.ncols;
    const unsigned rb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
    hipLaunchKernelGGL(k_cs_part_reduce<T>, dim3(rb), dim3(256), 0, st, k, c.ncols, ndies,
                       (const T *)part, Y, ldy);
    return hipGetLastError();
  }
  }
  if (nbt > 1)  // bucket tiles re-read A: ordinary loads, so the die's L2 keeps it
    return vec ? launch_cs_xcd_k<T, NT, true, SRC, UNR, false, false>(
                     grid, lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, Y, ldy,
                     status)
               : launch_cs_xcd_k<T, NT, false, SRC, UNR, false, false>(
                     grid, lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, Y, ldy,
                     status);
  return vec ? launch_cs_xcd_k<T, NT, true, SRC, UNR, true, false>(
                   grid, lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, Y, ldy,
                   status)
             : launch_cs_xcd_k<T, NT, false, SRC, UNR, true, false>(
                   grid, lds, st, d, c, code, h, s, k, ktile, nct, nbt, xcds, spx, rpx, Y, ldy,
                   status);
}

template <typename T, int NT, int SRC>
static hipError_t launch_cs_lds_v(bool vec, dim3 grid, size_t lds, hipStream_t st, int64_t d,
                                  const Cols<T> &c, const uint32_t *code, const int32_t *h,
                                  const int8_t *s, int64_t k, int64_t ktile, int64_t rows, T *Y,
                                  int64_t ldy, int *status) {
  const void *fn = vec ? (const void *)k_cs_lds<T, NT, true, SRC>
                       : (const void *)k_cs_lds<T, NT, false, SRC>;
  hipError_t e = allow_dynamic_lds(fn, (int)lds);
  if (e != hipSuccess) return e;
  if (vec)
    hipLaunchKernelGGL((k_cs_lds<T, NT, true, SRC>), grid, dim3(1024), lds, st, d, c, code, h, s,
                       k, ktile, rows, Y, ldy, status);
  else
    hipLaunchKernelGGL((k_cs_lds<T, NT, false, SRC>), grid, dim3(1024), lds, st, d, c, code, h,
                       s, k, ktile, rows, Y, ldy, status);
  return hipGetLastError();
}

template <typename T, int NT>
static hipError_t launch_cs_lds_nt(bool vec, dim3 grid, size_t lds, hipStream_t st, int64_t d,
                                   const Cols<T> &c, const uint32_t *code, const int32_t *h,
                                   const int8_t *s, int64_t k, int64_t ktile, int64_t rows, T *Y,
                                   int64_t ldy, int *status) {
  if (c.hashed) return hipErrorNotSupported;  // the persistent schedule only
  if (code)
    return launch_cs_lds_v<T, NT, kSrcCode>(vec, grid, lds, st, d, c, code, h, s, k, ktile, rows,
                                            Y, ldy, status);
  return launch_cs_lds_v<T, NT, kSrcHS>(vec, grid, lds, st, d, c, code, h, s, k, ktile, rows, Y,
                                        ldy, status);
}

// h and s of the hash-generated sketch, materialised (rows i of [0, d)).
__global__ void k_hash_sketch(int64_t d, int64_t k, uint64_t key, int32_t *__restrict__ h,
                              int8_t *__restrict__ s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t w = hash_word(key, i, k);
    h[i] = (int32_t)(w & kIdxMask);
    s[i] = (w & kSignBit) ? (int8_t)-1 : (int8_t)1;
  }
}

hipError_t launch_hash_sketch(int64_t d, int64_t k, uint64_t key, int32_t *h, int8_t *s,
                              hipStream_t st) {
  if (d <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((d + 255) / 256, 8192);
  hipLaunchKernelGGL(k_hash_sketch, dim3(blocks), dim3(256), 0, st, d, k, key, h, s);
  return hipGetLastError();
}

// LDS CountSketch.  Default: the persistent die-aware schedule; the earlier
// one-workgroup-per-(chunk, tile) grid is kept behind MS_CS_GRID (tuning).
template <typename T>
hipError_t launch_cs_lds(int64_t d, int64_t k, const Cols<T> &c, const uint32_t *code,
                         const int32_t *h, const int8_t *s, T *Y, int64_t ldy, bool zero_first,
                         int *status, hipStream_t st, const CsTuning *tune, void *part,
                         size_t part_bytes) {
  hipError_t e = zero_first ? launch_fill_zero<T>(Y, k, c.ncols, ldy, st) : hipSuccess;
  if (e != hipSuccess || d <= 0 || c.ncols <= 0) return e;
  const DevInfo &di = dev_info();
  const int64_t w = 8;  // bytes of an LDS partial-sum slot (FP64 for both data types)
  const int64_t wd = sizeof(T);
  const int64_t cap = std::min<int64_t>(di.lds_per_block, 128 * 1024);
  int64_t ktile = k;
  if (k * w > cap) {
    ktile = 1;
    while (ktile * 2 * w <= cap) ktile *= 2;
  }
  const int64_t nbt = (k + ktile - 1) / ktile;
  // the data columns need only element alignment (Vec16); the codes, or h
  // and s, are loaded W rows at a time at multiples of W
  const uintptr_t mis = reinterpret_cast<uintptr_t>(code) | reinterpret_cast<uintptr_t>(h);
  const uintptr_t smis = reinterpret_cast<uintptr_t>(s) & (uintptr_t)(16 / wd - 1);
  const bool vec = (mis & 15) == 0 && smis == 0;
  const bool grid_variant = tune && tune->grid_variant;
  if (!grid_variant) {
    const int xcds = (di.cus % di.xcds == 0) ? di.xcds : 1;
    int64_t rpx = (d + xcds - 1) / xcds;
    rpx = (rpx + 255) / 256 * 256;
    // columns per workgroup: as many as LDS holds (and the caller allows)
    // while each workgroup still streams at least 8 rows per flushed bucket
    auto spx_of = [&](int nt_) {
      const int64_t l = ktile * w * nt_;
      return di.cus / xcds * (int)std::max<int64_t>(1, std::min<int64_t>(2, di.lds_per_block / l));
    };
    int nt = 1;
    const int want_nt = tune && tune->cols_per_wg ? tune->cols_per_wg : 8;
    while (nt * 2 <= want_nt && ktile * w * nt * 2 <= cap && nt * 2 <= c.ncols) {
      const int64_t nct2 = (c.ncols + nt * 2 - 1) / (nt * 2);
      const int64_t per_wg = nct2 * nbt * rpx / std::max(1, spx_of(nt * 2));
      if (!(tune && tune->cols_per_wg) && per_wg < 8 * ktile * nbt) break;
      nt *= 2;
    }
    const int64_t lds = ktile * w * nt;
    const int spx = spx_of(nt);
    if (nbt > spx) return hipErrorNotSupported;
    const int64_t nct = (c.ncols + nt - 1) / nt;
    const int grid = xcds * spx;
    // the per-die partial schedule, when the caller's buffer holds it and the
    // device is the one its shape was chosen for
    const size_t need = cs_part_bytes(d, k, c.ncols, wd);
    T *pb = (part && need && part_bytes >= need && xcds == 8 && spx == 32 && nt == 1)
                ? static_cast<T *>(part)
                : nullptr;
#define MS_XCD_CASE(NT_)                                                                         \
  if (nt == NT_)                                                                                 \
    return c.hashed ? launch_cs_xcd_v<T, NT_, kSrcHash>(vec, grid, lds, st, d, c, code, h, s, k,  \
                                                        ktile, (int)nct, (int)nbt, xcds, spx,    \
                                                        rpx, Y, ldy, pb, status)                 \
           : code   ? launch_cs_xcd_v<T, NT_, kSrcCode>(vec, grid, lds, st, d, c, code, h, s, k,  \
                                                        ktile, (int)nct, (int)nbt, xcds, spx,    \
                                                        rpx, Y, ldy, pb, status)                 \
                    : launch_cs_xcd_v<T, NT_, kSrcHS>(vec, grid, lds, st, d, c, code, h, s, k,    \
                                                      ktile, (int)nct, (int)nbt, xcds, spx, rpx, \
                                                      Y, ldy, pb, status);
    MS_XCD_CASE(8)
    MS_XCD_CASE(4)
    MS_XCD_CASE(2)
    MS_XCD_CASE(1)
#undef MS_XCD_CASE
    return hipErrorInvalidValue;
  }
  // grid variant: one workgroup per (row chunk, column tile, bucket tile)
  const int64_t lds1 = ktile * w;
  const int64_t c_hi = std::max<int64_t>(1, d / 2048);
  int nt = 1;
  while (nt < 8 && lds1 * nt * 2 <= cap && nt * 2 <= c.ncols) {
    const int64_t units2 = ((c.ncols + nt * 2 - 1) / (nt * 2)) * nbt;
    const int64_t per_cu2 = std::max<int64_t>(1, std::min<int64_t>(2, di.lds_per_block / (lds1 * nt * 2)));
    if (units2 * c_hi < (int64_t)di.cus * per_cu2) break;
    nt *= 2;
  }
  const int64_t nct = (c.ncols + nt - 1) / nt;
  const int64_t lds = lds1 * nt;
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(2, di.lds_per_block / lds));
  const int64_t slots = (int64_t)di.cus * per_cu;
  const int64_t units = nct * nbt;
  const int64_t c_flush = std::max<int64_t>(1, d / (16 * ktile));
  int64_t chunks = std::min(c_hi, std::max(c_flush, (slots + units - 1) / units));
  const int64_t rounds = std::max<int64_t>(1, (units * chunks + slots / 2) / slots);
  chunks = std::max<int64_t>(1, std::min(c_hi, rounds * slots / units));
  int64_t rows = (d + chunks - 1) / chunks;
  rows = (rows + 255) / 256 * 256;
  chunks = (d + rows - 1) / rows;
  const dim3 grid((unsigned)chunks, (unsigned)nct, (unsigned)nbt);
  switch (nt) {
    case 8: return launch_cs_lds_nt<T, 8>(vec, grid, lds, st, d, c, code, h, s, k, ktile, rows, Y, ldy, status);
    case 4: return launch_cs_lds_nt<T, 4>(vec, grid, lds, st, d, c, code, h, s, k, ktile, rows, Y, ldy, status);
    case 2: return launch_cs_lds_nt<T, 2>(vec, grid, lds, st, d, c, code, h, s, k, ktile, rows, Y, ldy, status);
    default: return launch_cs_lds_nt<T, 1>(vec, grid, lds, st, d, c, code, h, s, k, ktile, rows, Y, ldy, status);
  }
}
template hipError_t launch_cs_lds<double>(int64_t, int64_t, const Cols<double> &, const uint32_t *,
                                          const int32_t *, const int8_t *, double *, int64_t, bool,
                                          int *, hipStream_t, const CsTuning *, void *, size_t);
template hipError_t launch_cs_lds<float>(int64_t, int64_t, const Cols<float> &, const uint32_t *,
                                         const int32_t *, const int8_t *, float *, int64_t, bool,
                                         int *, hipStream_t, const CsTuning *, void *, size_t);

// ------------------------------------------------------------------ sorted (deterministic)

// One thread per (bucket, column): the bucket's rows, in ascending row order
// (sperm from the stable plan), are folded into +0.0 one after the other --
// exactly the sequential order of Alg. 2, so the result is bit-identical to
// it.  Loads are issued four ahead of the dependent adds.
template <typename T>
__global__ __launch_bounds__(256) void k_cs_sorted(int64_t k, Cols<T> cols,
                                                   const int32_t *__restrict__ off,
                                                   const uint32_t *__restrict__ sperm,
                                                   T *__restrict__ Y, int64_t ldy) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (b >= k) return;
  const T *cp = col_ptr(cols, c);
  const int32_t j0 = off[b], j1 = off[b + 1];
  T y = T(0);
  int32_t j = j0;
  for (; j + 4 <= j1; j += 4) {
    const uint32_t e0 = sperm[j], e1 = sperm[j + 1], e2 = sperm[j + 2], e3 = sperm[j + 3];
    const T a0 = cp[e0 & kIdxMask], a1 = cp[e1 & kIdxMask], a2 = cp[e2 & kIdxMask],
            a3 = cp[e3 & kIdxMask];
    y = y + apply_sign(a0, e0);
    y = y + apply_sign(a1, e1);
    y = y + apply_sign(a2, e2);
    y = y + apply_sign(a3, e3);
  }
  for (; j < j1; ++j) {
    const uint32_t e = sperm[j];
    y = y + apply_sign(cp[e & kIdxMask], e);
  }
  Y[b + (int64_t)c * ldy] = y;
}

template <typename T>
hipError_t launch_cs_sorted(int64_t k, const Cols<T> &c, const int32_t *off,
                            const uint32_t *sperm, T *Y, int64_t ldy, hipStream_t st) {
  if (c.ncols <= 0) return hipSuccess;
  for (int c0 = 0; c0 < c.ncols; c0 += 65535) {
    Cols<T> sub = c;
    const int nc = std::min(65535, c.ncols - c0);
    if (c0 < c.n_a) {
      sub.A = c.A + (int64_t)c0 * c.lda;
      sub.n_a = c.n_a - c0;
    } else {
      sub.A = nullptr;
      sub.B = c.B + (int64_t)(c0 - c.n_a) * c.ldb;
      sub.n_a = 0;
    }
    sub.ncols = nc;
    hipLaunchKernelGGL(k_cs_sorted<T>, dim3((unsigned)((k + 255) / 256), nc), dim3(256), 0, st, k,
                       sub, off, sperm, Y + (int64_t)c0 * ldy, ldy);
  }
  return hipGetLastError();
}
template hipError_t launch_cs_sorted<double>(int64_t, const Cols<double> &, const int32_t *,
                                             const uint32_t *, double *, int64_t, hipStream_t);
template hipError_t launch_cs_sorted<float>(int64_t, const Cols<float> &, const int32_t *,
                                            const uint32_t *, float *, int64_t, hipStream_t);

}  // namespace ms
