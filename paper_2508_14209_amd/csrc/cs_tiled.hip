// cs_tiled.hip -- CountSketch Y += S [A | B] (Def. 3, Eq. (2), Alg. 2) when
// the bucket partial sums of one column do not fit in one workgroup's LDS
// (k > 16384 FP64 slots), e.g. k = 32,768 or 131,072 buckets.
//
// The buckets are split into nbt tiles of ktile buckets; tile t's partial
// sums live in the LDS of the workgroups that own tile t.  A plain tiled
// scheme lets every tile's workgroup stream every row and keep the rows of
// its tile, so each row is decoded and issues a (masked) LDS atomic nbt
// times.  Here a plan, built once per call from the rows' buckets, groups
// the rows of every block of 8192 consecutive rows by tile (a stable
// counting sort inside the block): entry = row offset in the block (13 bits)
// | bucket within the tile (15 bits) | sign bit.  Tile t's workgroup then
// visits only its own entries: it reads the entry, gathers that row's value
// from the column (the rows of an entry list ascend, so a wave's gathers fall
// in a few cache lines) and adds it to LDS.  Every element is decoded and
// added once, as in Alg. 2.
//
// Schedule: one workgroup per compute unit (the partial sums of a tile take
// up to 160 KB of LDS), workgroup g on die g % 8.  On each die the
// workgroups form groups of nbt, one per tile; a group walks a contiguous
// share of the (column, row block) space, so the nbt members read the same
// cache lines of A at about the same time through their die's L2.  A
// workgroup adds its partial sums to Y (device atomics) when its share
// leaves a column.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

constexpr int kBlkLog2 = 13;                   // rows per plan block: 8192
constexpr int64_t kBlk = (int64_t)1 << kBlkLog2;
constexpr uint32_t kOffMask = (uint32_t)kBlk - 1;
constexpr int kLbShift = kBlkLog2;             // bucket within the tile: bits 13..27
constexpr uint32_t kLbMask = 0x7fffu;
constexpr int64_t kMaxSlots = 20480;           // FP64 partial sums in 160 KB of LDS
constexpr int kMaxTiles = 32;                  // at least one group per die of 32 CUs
constexpr int kPlanThreads = 1024;             // 8 rows per thread in a plan block
constexpr int kUnits = 8;                      // (column, block) units per batch
constexpr int kPer = 4;                        // gathers in flight per thread

struct TileShape {
  int nbt = 0;  // 0: not applicable
  int64_t ktile = 0, nblk = 0;
};

TileShape tile_shape(int64_t d, int64_t k) {
  TileShape s;
  if (d < 1 || k <= 16384) return s;
  int64_t need = (k + kMaxSlots - 1) / kMaxSlots;
  int nbt = 2;
  while (nbt < need) nbt *= 2;
  // two bucket tiles: the untiled kernel, whose two tiles each stream every
  // row, measured faster (16,777,216 x 129 FP32, k = 32,768: 2.98 vs 3.2 ms);
  // from four tiles the per-tile entry lists win (k = 131,072: 6.0 vs 7.9 ms)
  if (nbt < 4 || nbt > kMaxTiles) return s;
  s.nbt = nbt;
  s.ktile = (k + nbt - 1) / nbt;
  s.nblk = (d + kBlk - 1) / kBlk;
  return s;
}

// Per block: the valid rows' entries, tile by tile, each tile's rows
// ascending (thread i holds rows 8i .. 8i+7 of the block).  boff[b*(nbt+1)+t]
// = first entry of tile t in the block, boff[b*(nbt+1)+nbt] = valid rows.
// SRC as in the LDS CountSketch: stored h and s (checked here), or packed
// codes from ms_pack_sketch.
template <bool CODE>
__global__ __launch_bounds__(kPlanThreads) void k_tile_plan(
    int64_t d, int64_t k, int64_t ktile, int nbt, int64_t nblk, const uint32_t *__restrict__ code,
    const int32_t *__restrict__ h, const int8_t *__restrict__ s, uint32_t *__restrict__ ent,
    int32_t *__restrict__ boff, int *status) {
  __shared__ int32_t wave_sum[kPlanThreads / 64];
  __shared__ int32_t tile_base_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool bad = false;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * kBlk;
    const int64_t rows = min(kBlk, d - r0);
    uint32_t w[8];   // entry without the offset field set; 0xffffffff: invalid / absent
    int tl[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t r = (int64_t)tid * 8 + q;
      tl[q] = -1;
      w[q] = 0xffffffffu;
      if (r < rows) {
        uint32_t b;
        uint32_t sg;
        bool ok;
        if (CODE) {
          const uint32_t e = code[r0 + r];
          b = e & kIdxMask;
          sg = e & kSignBit;
          ok = (int64_t)b < k;
        } else {
          const int32_t hb = h[r0 + r];
          const int8_t sv = s[r0 + r];
          b = (uint32_t)hb;
          sg = sv < 0 ? kSignBit : 0u;
          ok = ((uint32_t)hb < (uint32_t)k) & ((sv == 1) | (sv == -1));
        }
        bad |= !ok;
        if (ok) {
          const uint32_t t = b / (uint32_t)ktile;
          tl[q] = (int)t;
          w[q] = (uint32_t)r | ((b - t * (uint32_t)ktile) << kLbShift) | sg;
        }
      }
    }
    if (tid == 0) tile_base_s = 0;
    __syncthreads();
    for (int t = 0; t < nbt; ++t) {
      int c = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) c += tl[q] == t;
      // exclusive scan of c over the workgroup (thread order = row order)
      int incl = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane == 63) wave_sum[wave] = incl;
      __syncthreads();
      int before = tile_base_s;
      for (int v = 0; v < wave; ++v) before += wave_sum[v];
      int pos = before + incl - c;
      if (tid == 0) boff[blk * (nbt + 1) + t] = tile_base_s;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (tl[q] == t) ent[r0 + pos++] = w[q];
      __syncthreads();
      if (tid == kPlanThreads - 1) tile_base_s = pos;
      __syncthreads();
    }
    if (tid == 0) boff[blk * (nbt + 1) + nbt] = tile_base_s;
    __syncthreads();
  }
  if (bad) record_status(status, MS_ERR_RANGE);
}

template <typename T>
__device__ __forceinline__ const T *tcol(const Cols<T> &c, int j) {
  return j < c.n_a ? c.A + (int64_t)j * c.lda : c.B + (int64_t)(j - c.n_a) * c.ldb;
}

// Add the LDS partial sums of column c (buckets t*ktile + l, l < kt) to Y and
// clear them.
template <typename T>
__device__ __forceinline__ void tiled_flush(double *acc, uint32_t kt, int64_t bbase, int c,
                                            T *__restrict__ Y, int64_t ldy) {
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < kt; l += blockDim.x) {
    const double v = acc[l];
    acc[l] = 0.0;
    if (v != 0.0) unsafeAtomicAdd(&Y[bbase + l + (int64_t)c * ldy], (T)v);
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_cs_tiled(int64_t d, Cols<T> cols, int64_t k,
                                                   int64_t ktile, int nbt, int64_t nblk,
                                                   const uint32_t *__restrict__ ent,
                                                   const int32_t *__restrict__ boff, int xcds,
                                                   int subs, T *__restrict__ Y, int64_t ldy) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);
  const int g = blockIdx.x;
  const int x = g % xcds, slot = g / xcds;
  if (slot >= subs * nbt) return;
  const int t = slot % nbt, sub = slot / nbt;
  const int64_t ngroups = (int64_t)subs * xcds;
  const int64_t grp = (int64_t)sub * xcds + x;
  const int64_t bbase = (int64_t)t * ktile;
  if (bbase >= k) return;
  const uint32_t kt = (uint32_t)min(ktile, k - bbase);
  for (uint32_t l = threadIdx.x; l < kt; l += blockDim.x) acc[l] = 0.0;
  __syncthreads();
  const int64_t total = (int64_t)cols.ncols * nblk;
  int64_t u = total * grp / ngroups;
  const int64_t u1 = total * (grp + 1) / ngroups;
  int cur = -1;
  while (u < u1) {
    const int c = (int)(u / nblk);
    const int64_t b0 = u - (int64_t)c * nblk;
    const int64_t nb = min<int64_t>(kUnits, min(u1 - u, nblk - b0));
    if (c != cur) {
      if (cur >= 0) tiled_flush<T>(acc, kt, bbase, cur, Y, ldy);
      cur = c;
    }
    const T *col = tcol(cols, c);
    // the batch's entry lists, concatenated: unit j holds virtual positions
    // [pre[j], pre[j+1])
    int32_t e0[kUnits], pre[kUnits + 1];
    pre[0] = 0;
#pragma unroll
    for (int j = 0; j < kUnits; ++j) {
      int32_t a = 0, z = 0;
      if (j < nb) {
        const int32_t *bo = boff + (b0 + j) * (nbt + 1) + t;
        a = bo[0];
        z = bo[1];
      }
      e0[j] = a;
      pre[j + 1] = pre[j] + (z - a);
    }
    const int32_t L = pre[kUnits];
    for (int32_t base = 0; base < L; base += kPer * (int32_t)blockDim.x) {
      uint32_t e[kPer];
      int64_t rb[kPer];
#pragma unroll
      for (int p = 0; p < kPer; ++p) {
        const int32_t v = base + p * (int32_t)blockDim.x + (int32_t)threadIdx.x;
        e[p] = 0xffffffffu;
        rb[p] = 0;
        if (v < L) {
          // the unit holding v: the last j with pre[j] <= v (static indices
          // only, so the small arrays stay in registers)
          int j = 0;
          int32_t ej = e0[0], pj = 0;
#pragma unroll
          for (int q = 1; q < kUnits; ++q)
            if (v >= pre[q]) {
              j = q;
              ej = e0[q];
              pj = pre[q];
            }
          const int64_t blk = b0 + j;
          e[p] = gload(ent + blk * kBlk + ej + (v - pj));
          rb[p] = blk * kBlk;
        }
      }
      T a[kPer];
#pragma unroll
      for (int p = 0; p < kPer; ++p)
        a[p] = e[p] != 0xffffffffu ? gload(col + rb[p] + (e[p] & kOffMask)) : T(0);
#pragma unroll
      for (int p = 0; p < kPer; ++p)
        if (e[p] != 0xffffffffu)
          atomicAdd(&acc[(e[p] >> kLbShift) & kLbMask], (double)apply_sign(a[p], e[p]));
    }
    u += nb;
  }
  if (cur >= 0) tiled_flush<T>(acc, kt, bbase, cur, Y, ldy);
}

}  // namespace

size_t cs_tile_plan_bytes(int64_t d, int64_t k) {
  const TileShape s = tile_shape(d, k);
  if (!s.nbt) return 0;
  return align_up((size_t)s.nblk * kBlk * 4) + align_up((size_t)s.nblk * (s.nbt + 1) * 4);
}

bool cs_tiled_supported(int64_t d, int64_t k) {
  const TileShape s = tile_shape(d, k);
  if (!s.nbt) return false;
  const DevInfo &di = dev_info();
  return di.lds_per_block >= s.ktile * 8 && di.cus % di.xcds == 0 && di.cus / di.xcds >= s.nbt;
}

hipError_t launch_tile_plan(int64_t d, int64_t k, const uint32_t *code, const int32_t *h,
                            const int8_t *s, void *plan, int *status, hipStream_t st) {
  const TileShape sh = tile_shape(d, k);
  if (!sh.nbt) return hipErrorInvalidValue;
  uint32_t *ent = static_cast<uint32_t *>(plan);
  int32_t *boff = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(plan) +
                                              align_up((size_t)sh.nblk * kBlk * 4));
  const unsigned grid = (unsigned)std::min<int64_t>(sh.nblk, 4096);
  if (code)
    hipLaunchKernelGGL(k_tile_plan<true>, dim3(grid), dim3(kPlanThreads), 0, st, d, k, sh.ktile,
                       sh.nbt, sh.nblk, code, nullptr, nullptr, ent, boff, status);
  else
    hipLaunchKernelGGL(k_tile_plan<false>, dim3(grid), dim3(kPlanThreads), 0, st, d, k, sh.ktile,
                       sh.nbt, sh.nblk, nullptr, h, s, ent, boff, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cs_tiled(int64_t d, int64_t k, const Cols<T> &c, const void *plan, T *Y,
                           int64_t ldy, hipStream_t st) {
  const TileShape sh = tile_shape(d, k);
  if (!sh.nbt) return hipErrorInvalidValue;
  if (c.ncols <= 0) return hipSuccess;
  const DevInfo &di = dev_info();
  const int xcds = di.xcds;
  const int subs = di.cus / xcds / sh.nbt;
  const size_t lds = (size_t)sh.ktile * 8;
  const void *fn = (const void *)k_cs_tiled<T>;
  hipError_t e = allow_dynamic_lds(fn, (int)lds);
  if (e != hipSuccess) return e;
  const uint32_t *ent = static_cast<const uint32_t *>(plan);
  const int32_t *boff = reinterpret_cast<const int32_t *>(
      static_cast<const unsigned char *>(plan) + align_up((size_t)sh.nblk * kBlk * 4));
  hipLaunchKernelGGL(k_cs_tiled<T>, dim3((unsigned)(xcds * subs * sh.nbt)), dim3(1024), lds, st,
                     d, c, k, sh.ktile, sh.nbt, sh.nblk, ent, boff, xcds, subs, Y, ldy);
  return hipGetLastError();
}
template hipError_t launch_cs_tiled<double>(int64_t, int64_t, const Cols<double> &, const void *,
                                            double *, int64_t, hipStream_t);
template hipError_t launch_cs_tiled<float>(int64_t, int64_t, const Cols<float> &, const void *,
                                           float *, int64_t, hipStream_t);

}  // namespace ms
