// gemm.hip -- the Gaussian stage Z = G Y of the multisketch S2(S1 x)
// (Sec. 1 of Higgins, Boman, Yamazaki, arXiv 2508.14209; Table 1), on the
// gfx950 matrix cores.
//
// Shapes are short and wide in K: M = k2 (2n), N = n + nrhs, K = k (2n^2).
// The K dimension is split across workgroups; each writes a partial M x N
// block and a second kernel adds the partials in a fixed order (four
// consecutive runs of splits, each in split order, then the four run sums in
// order), so the result does not depend on scheduling.  A 16-bit G uses
// 256 x 144 output tiles staged through LDS; FP64 and FP32 use 64 x 64 tiles
// with fragments loaded straight from memory.
//
// Matrix-core instructions (one 16x16 output block per instruction):
//   FP64: v_mfma_f64_16x16x4_f64       (K step 4)
//   FP32: v_mfma_f32_16x16x4_f32       (K step 4)
//   BF16: v_mfma_f32_16x16x32_bf16     (K step 32, FP32 accumulation)
//   FP16: v_mfma_f32_16x16x32_f16      (K step 32, FP32 accumulation)
// Operand layout per lane l (64 lanes): A element (row l%16, k-group l/16),
// B element (k-group l/16, column l%16).  The four accumulator values r of
// lane l belong to column l%16 and to row 4*(l/16)+r for the FP32 and BF16
// instructions, but to row (l/16)+4*r for the FP64 one (measured).
#include <algorithm>

#include "ms_internal.h"

namespace ms {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8u16 __attribute__((ext_vector_type(8)));
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest, ties to even (NaN kept quiet).
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0u)
    return (unsigned short)((u | 0x00400000u) >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Two FP32 values rounded to nearest-even BF16, packed (first in the low
// half): the hardware conversion, which agrees with f32_to_bf16_rne on
// every finite value.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2_rne(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

// Two FP32 values rounded to nearest-even FP16, packed (first in the low half).
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
__device__ __forceinline__ uint32_t f16x2_rne(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, f16x2_t));
}

enum { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_F16 = 3 };

template <int DT>
struct Mf;
template <>
struct Mf<DT_F64> {
  using TG = double;
  using TY = double;
  using Acc = double;
  using Frag = double;
  using AccV = v4d;
  static constexpr int KS = 4;
  __device__ static AccV mma(Frag a, Frag b, AccV c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int out_row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct Mf<DT_F32> {
  using TG = float;
  using TY = float;
  using Acc = float;
  using Frag = float;
  using AccV = v4f;
  static constexpr int KS = 4;
  __device__ static AccV mma(Frag a, Frag b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int out_row(int lk, int r) { return 4 * lk + r; }
};
// The 16-bit formats of the LDS-staged tile: conversion of FP32 pairs,
// the value of a converted half as FP32, and the matrix-core product.
template <int DT>
struct Half16;
template <>
struct Half16<DT_BF16> {
  using V8 = v8bf;
  __device__ static uint32_t pack2(float lo, float hi) { return bf16x2_rne(lo, hi); }
  __device__ static float lo_f32(uint32_t w) { return __uint_as_float(w << 16); }
  __device__ static float hi_f32(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
  __device__ static v4f mma(V8 a, V8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Half16<DT_F16> {
  using V8 = v8h;
  __device__ static uint32_t pack2(float lo, float hi) { return f16x2_rne(lo, hi); }
  __device__ static float lo_f32(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
  }
  __device__ static float hi_f32(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
  }
  __device__ static v4f mma(V8 a, V8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// A fragment: G rows [row], k-group starting at kq (KS/4 consecutive k).
template <int DT>
__device__ __forceinline__ typename Mf<DT>::Frag load_a(const typename Mf<DT>::TG *G, int64_t ldg,
                                                        int M, int row, int64_t kq, int64_t ke);
template <>
__device__ __forceinline__ double load_a<DT_F64>(const double *G, int64_t ldg, int M, int row,
                                                 int64_t kq, int64_t ke) {
  return (row < M && kq < ke) ? gload(G + row + kq * ldg) : 0.0;
}
template <>
__device__ __forceinline__ float load_a<DT_F32>(const float *G, int64_t ldg, int M, int row,
                                                int64_t kq, int64_t ke) {
  return (row < M && kq < ke) ? gload(G + row + kq * ldg) : 0.0f;
}

// B fragment: Y column [col], k-group starting at kq.
template <int DT>
__device__ __forceinline__ typename Mf<DT>::Frag load_b(const typename Mf<DT>::TY *Y, int64_t ldy,
                                                        int N, int col, int64_t kq, int64_t ke);
template <>
__device__ __forceinline__ double load_b<DT_F64>(const double *Y, int64_t ldy, int N, int col,
                                                 int64_t kq, int64_t ke) {
  return (col < N && kq < ke) ? Y[kq + (int64_t)col * ldy] : 0.0;
}
template <>
__device__ __forceinline__ float load_b<DT_F32>(const float *Y, int64_t ldy, int N, int col,
                                                int64_t kq, int64_t ke) {
  return (col < N && kq < ke) ? Y[kq + (int64_t)col * ldy] : 0.0f;
}

// Workgroup = 4 waves over a 64 x 64 output tile (each wave 32 x 32, i.e.
// 2 x 2 matrix-core blocks), one K chunk per workgroup.  Fragments are loaded U instructions ahead: the loads of the next batch are
// in flight while the current batch runs on the matrix cores.

// One 64 x 64 output tile (m_tile, n_tile) of G[:, kb:ke] Y[kb:ke, :], written
// to P (ld M) -- the body shared by the single-problem and batched kernels.
template <int DT>
__device__ __forceinline__ void gemm_tile(int M, int N, const typename Mf<DT>::TG *__restrict__ G,
                                          int64_t ldg, const typename Mf<DT>::TY *__restrict__ Y,
                                          int64_t ldy, typename Mf<DT>::Acc *__restrict__ P,
                                          int64_t kb, int64_t ke, int m_tile, int n_tile) {
  using F = Mf<DT>;
  constexpr int U = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int m_base = m_tile * 64 + (wave & 1) * 32;
  const int n_base = n_tile * 64 + (wave >> 1) * 32;
  constexpr int KPL = F::KS / 4;  // k values per lane per instruction
  typename F::AccV acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = typename F::AccV{};
  typename F::Frag a[U][2], b[U][2];
  auto load_batch = [&](int64_t k0, typename F::Frag (&fa)[U][2], typename F::Frag (&fb)[U][2]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kq = k0 + (int64_t)u * F::KS + (int64_t)lk * KPL;
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[u][i] = load_a<DT>(G, ldg, M, m_base + 16 * i + li, kq, ke);
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[u][j] = load_b<DT>(Y, ldy, N, n_base + 16 * j + li, kq, ke);
    }
  };
  load_batch(kb, a, b);
  for (int64_t kk = kb; kk < ke; kk += (int64_t)F::KS * U) {
    typename F::Frag an[U][2], bn[U][2];
    const bool more = kk + (int64_t)F::KS * U < ke;
    if (more) load_batch(kk + (int64_t)F::KS * U, an, bn);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = F::mma(a[u][i], b[u][j], acc[i][j]);
    if (more) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[u][i] = an[u][i];
          b[u][i] = bn[u][i];
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n_base + 16 * j + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m_base + 16 * i + F::out_row(lk, r);
        if (row < M && col < N) P[row + (int64_t)col * M] = acc[i][j][r];
      }
    }
}

// ------------------------------------------------------------ wide 16-bit tiles
// The BF16 / FP16 stage with 256 x 144 output tiles: four waves (one per
// SIMD), wave w owning rows 64 w .. 64 w + 63 of the tile and all 144 columns
// (4 x 9 blocks of 16 x 16, 144 accumulator registers).  K advances in stages
// of 32: per stage the workgroup stages G's 256 x 32 tile (loaded as 16-byte
// runs of 8 rows at one k, written to LDS k-contiguous per row) and Y's
// 32 x 144 tile (FP32, split into YT 16-bit terms on the way in); up to three
// stages of global loads are in flight while one is on the matrix cores.
// With 64 x 64 tiles every element of G would be fetched by ceil(N/64)
// workgroups and every element of Y by ceil(M/64); here by ceil(N/144) and
// ceil(M/256) (once each for M <= 256 and N <= 144: every sketch of the
// serving workload).  The k steps of a K chunk run in ascending order and
// the terms of a step small first.
//
// LDS: G's tile row R starts at element 40 R + 32 (R / 8): rows padded to 40
// elements (fragment reads of 16 lanes hit distinct banks), and each 8-row
// group shifted by 16 banks so that the transposing 4-byte writes of a wave
// (16 k pairs x 4 row groups) cost two passes, not four.
//
// YT = 1: Y rounded to the 16-bit format (nearest even).  YT = 3: Y as the
// sum of three terms, hi = h(y), mid = h(y - hi), lo = h(y - hi - mid); each
// remainder is exact in FP32.  For BF16 (8-bit significand, FP32's exponent
// range) the last remainder fits BF16, so hi + mid + lo = y exactly for every
// normal FP32 y, and G Y is formed from the exact Y (G's values are BF16
// data) with three matrix-core products per step and FP32 accumulation:
// FP32-level accuracy at BF16 instruction rate, with G read once.
// FP16 (11-bit significand, largest finite 65504) first scales column c of Y
// by the power of two cs[2c] = 2^-e_c that brings its largest magnitude into
// [2^14, 2^15), and multiplies the column's result by cs[2c + 1] = 2^e_c;
// the three terms then hold y exactly down to 2^-40 of the column's largest
// magnitude (smaller parts of an entry fall below FP16's subnormals).
constexpr int kWTM = 256, kWTN = 144, kWKS = 32, kWPad = 40, kWThreads = 256;
constexpr int kWNB = kWTN / 16;                       // column blocks per tile
constexpr int kWAElems = kWTM * kWPad + (kWTM / 8) * 32;  // G tile incl. group shifts

__device__ __forceinline__ int wide_arow(int r) { return r * kWPad + (r >> 3) * 32; }

template <int YT>
constexpr int wide_stage_elems() {
  return kWAElems + YT * kWTN * kWPad;
}
template <int YT>
constexpr int wide_lds_bytes() {
  return 2 * wide_stage_elems<YT>() * 2;
}

// One stage's global loads held in registers: for G tasks v = 0, 1 the rows
// 8 g .. 8 g + 7 at k 2 kp and 2 kp + 1; Y columns and k octets of up to
// three tasks.
struct WideRegs {
  v8u16 g[2][2];
  float y[3][8];
};

// FAST: G's leading dimension a multiple of 8 and G 16-byte aligned, M a
// multiple of 8 (each 8-row group of a tile wholly inside or outside), Y's
// leading dimension a multiple of 4 and Y 16-byte aligned, K a multiple of
// 32 (every stage wholly inside K).  Then every load is a 16-byte load from a
// running pointer with no per-load condition: a row group or column outside
// the tile reads row 0 or column n0 instead (its products land in rows or
// columns that are never stored), and the fetches past the chunk's last stage
// re-read that stage (their stages are never computed).  Else every element
// is loaded alone, guarded, zero outside.
template <int DT, int YT, bool FAST>
__device__ __forceinline__ void gemm_tile_wide(int M, int N, const unsigned short *__restrict__ G,
                                               int64_t ldg, const float *__restrict__ Y,
                                               int64_t ldy, const float *__restrict__ cs,
                                               float *__restrict__ P, int64_t kb, int64_t ke,
                                               int64_t kstride, int m0, int n0,
                                               unsigned short *lds) {
  using H = Half16<DT>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // G task v: k pair kp (fastest), row group g
  const int kp = tid & 15;
  // Y task u (tid + 256 u): column / 4, k octet % 4; the third task for the
  // first wave only (a wave-uniform condition)
  const int ny = wave == 0 ? 3 : 2;
  const int64_t klen = ke - kb;
  float ysc[3] = {1.0f, 1.0f, 1.0f};
  if (DT == DT_F16) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int c = (tid + u * kWThreads) >> 2;
      if (u < ny && n0 + c < N) ysc[u] = cs[2 * (n0 + c)];
    }
  }
  const unsigned short *gp[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int rb = m0 + 8 * ((tid + v * kWThreads) >> 4);
    gp[v] = G + (rb < M ? rb : 0) + (kb + 2 * kp) * ldg;
  }
  const int64_t gstep = kstride * ldg;
  const float *yp[3];
  int ykq[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int t = tid + u * kWThreads;
    const int c = t >> 2;
    const bool cv = t < kWTN * 4 && n0 + c < N;
    ykq[u] = 8 * (t & 3);
    yp[u] = Y + kb + ykq[u] + (int64_t)(cv ? n0 + c : n0) * ldy;
  }
  int64_t krel = 0;  // start of the next stage to fetch, relative to kb
  auto fetch = [&](WideRegs &R) {
    if constexpr (FAST) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        R.g[v][0] = gload(reinterpret_cast<const v8u16 *>(gp[v]));
        R.g[v][1] = gload(reinterpret_cast<const v8u16 *>(gp[v] + ldg));
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        if (u >= ny) break;
        const v4f a = gload(reinterpret_cast<const v4f *>(yp[u]));
        const v4f b = gload(reinterpret_cast<const v4f *>(yp[u] + 4));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          R.y[u][e] = a[e];
          R.y[u][4 + e] = b[e];
        }
      }
      if (krel + kstride < klen) {  // the next stage exists (uniform)
#pragma unroll
        for (int v = 0; v < 2; ++v) gp[v] += gstep;
#pragma unroll
        for (int u = 0; u < 3; ++u) yp[u] += kstride;
      }
    } else {
      const int64_t k0 = kb + krel;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int rb = m0 + 8 * ((tid + v * kWThreads) >> 4);
        const int64_t kc = k0 + 2 * kp;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          R.g[v][0][r] = (kc < ke && rb + r < M) ? gload(G + rb + r + kc * ldg) : (unsigned short)0;
          R.g[v][1][r] = (kc + 1 < ke && rb + r < M) ? gload(G + rb + r + (kc + 1) * ldg)
                                                     : (unsigned short)0;
        }
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        if (u >= ny) break;
        const int t = tid + u * kWThreads;
        const int c = t >> 2;
        const int64_t kq = k0 + ykq[u];
        const bool cv = t < kWTN * 4 && n0 + c < N;
        const float *q = Y + kq + (int64_t)(cv ? n0 + c : n0) * ldy;
#pragma unroll
        for (int e = 0; e < 8; ++e) R.y[u][e] = (cv && kq + e < ke) ? gload(q + e) : 0.0f;
      }
    }
    krel += kstride;
  };
  auto lstore = [&](const WideRegs &R, int buf) {
    unsigned short *As = lds + buf * wide_stage_elems<YT>();
    unsigned short *Bs = As + kWAElems;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      // row r's word: its k = 2 kp value in the low half, k = 2 kp + 1 in the
      // high half; one byte permute per word (rows 2i and 2i + 1 share the
      // loaded words i)
      const int g = (tid + v * kWThreads) >> 4;
      const v4u32 w0 = __builtin_bit_cast(v4u32, R.g[v][0]);
      const v4u32 w1 = __builtin_bit_cast(v4u32, R.g[v][1]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        *reinterpret_cast<uint32_t *>(&As[wide_arow(8 * g + 2 * i) + 2 * kp]) =
            __builtin_amdgcn_perm(w1[i], w0[i], 0x05040100u);
        *reinterpret_cast<uint32_t *>(&As[wide_arow(8 * g + 2 * i + 1) + 2 * kp]) =
            __builtin_amdgcn_perm(w1[i], w0[i], 0x07060302u);
      }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      if (u >= ny) break;
      const int t = tid + u * kWThreads;
      if (t >= kWTN * 4) break;
      const int c = t >> 2, q8 = 8 * (t & 3);
      v4u32 bt[YT];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        float y0 = R.y[u][2 * p], y1 = R.y[u][2 * p + 1];
        if (DT == DT_F16) {
          y0 *= ysc[u];
          y1 *= ysc[u];
        }
#pragma unroll
        for (int tt = 0; tt < YT; ++tt) {
          const uint32_t w = H::pack2(y0, y1);
          bt[tt][p] = w;
          if (tt + 1 < YT) {
            y0 -= H::lo_f32(w);
            y1 -= H::hi_f32(w);
          }
        }
      }
#pragma unroll
      for (int tt = 0; tt < YT; ++tt)
        *reinterpret_cast<v4u32 *>(&Bs[(tt * kWTN + c) * kWPad + q8]) = bt[tt];
    }
  };
  // the wave's rows and the tile's block count are wave-uniform
  const int wrow = 64 * wave;
  const int nrow = min(4, (M - m0 - wrow + 15) / 16);  // 16-row blocks of the wave with rows
  const int nb = __builtin_amdgcn_readfirstlane(min(kWNB, (N - n0 + 15) / 16));
  v4f acc[4][kWNB];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < kWNB; ++j) acc[i][j] = v4f{};
  auto compute = [&](int buf) {
    if (nrow <= 0) return;
    const unsigned short *As = lds + buf * wide_stage_elems<YT>();
    const unsigned short *Bs = As + kWAElems;
    typename H::V8 a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *reinterpret_cast<const typename H::V8 *>(&As[wide_arow(wrow + 16 * i + li) + lk * 8]);
    // the stage's YT x 9 fragments of Y (small terms first, blocks in
    // order) in chunks of three: the next chunk's LDS reads are issued before
    // the current chunk's twelve products, and scheduling barriers keep that
    // order (unpinned, the compiler hoists every read and runs out of
    // registers)
    constexpr int kNF = YT * kWNB, kCH = 3;
    typename H::V8 bq[2][kCH];
    auto rd = [&](int f, typename H::V8 &dst) {
      const int tt = YT - 1 - f / kWNB, j = f % kWNB;
      dst = *reinterpret_cast<const typename H::V8 *>(
          &Bs[(tt * kWTN + 16 * j + li) * kWPad + lk * 8]);
    };
#pragma unroll
    for (int e = 0; e < kCH; ++e) rd(e, bq[0][e]);
#pragma unroll
    for (int c = 0; c < kNF / kCH; ++c) {
      if (c + 1 < kNF / kCH) {
#pragma unroll
        for (int e = 0; e < kCH; ++e) rd((c + 1) * kCH + e, bq[(c + 1) & 1][e]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < kCH; ++e) {
        const int j = (c * kCH + e) % kWNB;
        if (j < nb) {
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = H::mma(a[i], bq[c & 1][e], acc[i][j]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // Stages in pairs with no data-dependent condition around the loads (so
  // that the compiler keeps the younger stage's loads in flight across the
  // older one's LDS store): the fetches past the last stage load in-range
  // addresses, and a stage past the last is not computed.
  // NS register sets: NS - 1 stages of loads in flight (three on the fast
  // path, whose loads need few registers); stage s is in register set s % NS
  // and, once stored, in LDS buffer s % 2.
  constexpr int NS = FAST ? 4 : 2;
  const int64_t nst = (klen + kstride - 1) / kstride, ngroups = (nst + NS - 1) / NS;
  WideRegs R[NS];
#pragma unroll
  for (int i = 0; i < NS - 1; ++i) fetch(R[i]);
  lstore(R[0], 0);
  __syncthreads();
  for (int64_t q = 0; q < ngroups; ++q) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      fetch(R[(i + NS - 1) % NS]);           // stage q NS + i + NS - 1
      if (q * NS + i < nst) compute(i & 1);  // stage q NS + i
      lstore(R[(i + 1) % NS], (i + 1) & 1);  // stage q NS + i + 1
      __syncthreads();
    }
  }
  if (nrow <= 0) return;
#pragma unroll
  for (int j = 0; j < kWNB; ++j) {
    const int col = n0 + 16 * j + li;
    if (j >= nb || col >= N) continue;
    const float back = DT == DT_F16 ? cs[2 * col + 1] : 1.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row0 = m0 + wrow + 16 * i + 4 * lk;
      if (row0 >= M) continue;
      float *dst = P + row0 + (int64_t)col * M;
      v4f v = acc[i][j];
      if (DT == DT_F16) v = v * back;
      if ((M & 3) == 0 && row0 + 4 <= M) {
        *reinterpret_cast<v4f *>(dst) = v;
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row0 + r < M) dst[r] = v[r];
      }
    }
  }
}

// Workgroup g runs on die g % xcds; the tiles of one K chunk go to one die.
template <int DT, int YT, bool FAST>
__global__ __launch_bounds__(kWThreads) void k_gemm_wide(int M, int N, int64_t K,
                                                         const unsigned short *__restrict__ G,
                                                         int64_t ldg, const float *__restrict__ Y,
                                                         int64_t ldy, float *__restrict__ part,
                                                         int64_t kchunk, int tiles_m, int tiles,
                                                         int nsplit, int xcds,
                                                         const float *__restrict__ cs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = blockIdx.x;
  const int x = g % xcds, j = g / xcds;
  const int split = x + xcds * (j / tiles);
  if (split >= nsplit) return;
  const int tile = j % tiles;
  // contiguous K chunks (kchunk > 0) or, with kchunk = 0, K stages dealt
  // out in turn: split s takes stages s, s + nsplit, s + 2 nsplit, ...
  const int64_t kb = kchunk > 0 ? (int64_t)split * kchunk : (int64_t)split * kWKS;
  const int64_t ke = kchunk > 0 ? min(K, kb + kchunk) : K;
  const int64_t kstride = kchunk > 0 ? (int64_t)kWKS : (int64_t)kWKS * nsplit;
  gemm_tile_wide<DT, YT, FAST>(M, N, G, ldg, Y, ldy, cs, part + (int64_t)split * M * N, kb, ke,
                               kstride, (tile % tiles_m) * kWTM, (tile / tiles_m) * kWTN,
                               reinterpret_cast<unsigned short *>(smem_raw));
}

// Workgroup g runs on die g % xcds.  All output tiles of one K chunk are
// given to workgroups of the same die, so that chunk of G and Y is fetched
// from HBM into one L2 and the other tiles re-read it from there.
template <int DT>
__global__ __launch_bounds__(256) void k_gemm_splitk(int M, int N, int64_t K,
                                                     const typename Mf<DT>::TG *__restrict__ G,
                                                     int64_t ldg,
                                                     const typename Mf<DT>::TY *__restrict__ Y,
                                                     int64_t ldy,
                                                     typename Mf<DT>::Acc *__restrict__ part,
                                                     int64_t kchunk, int tiles_m, int tiles,
                                                     int nsplit, int xcds) {
  const int g = blockIdx.x;
  const int x = g % xcds, j = g / xcds;
  const int split = x + xcds * (j / tiles);
  if (split >= nsplit) return;
  const int tile = j % tiles;
  const int64_t kb = (int64_t)split * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  gemm_tile<DT>(M, N, G, ldg, Y, ldy, part + (int64_t)split * M * N, kb, ke, tile % tiles_m,
                tile / tiles_m);
}

// FP16 column scales: cs[2c] = 2^-e_c and cs[2c + 1] = 2^e_c with
// e_c = floor(log2 max_k |Y[k, c]|) - 14, so the scaled column's largest
// magnitude lies in [2^14, 2^15) (FP16's largest finite value is 65504).
// e_c is held in [-112, 112] (both factors normal FP32 numbers); a zero
// column, or one holding a NaN or an infinity, takes e_c = 0.  One workgroup
// per column.
__global__ __launch_bounds__(256) void k_f16_col_scale(int64_t K, const float *__restrict__ Y,
                                                       int64_t ldy, float *__restrict__ cs) {
  __shared__ float wmax[4];
  const int c = blockIdx.x;
  const float *y = Y + (int64_t)c * ldy;
  float m = 0.0f;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < K; i += blockDim.x) {
    const float v = fabsf(gload(y + i));
    bad |= !(v <= 3.4028235e38f);   // NaN or infinity
    m = fmaxf(m, v);
  }
  bad = __any(bad);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = bad ? -1.0f : m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float mm = 0.0f;
    bool anybad = false;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      anybad |= wmax[w] < 0.0f;
      mm = fmaxf(mm, wmax[w]);
    }
    int e = 0;
    if (!anybad && mm > 0.0f) e = min(112, max(-112, ilogbf(mm) - 14));
    cs[2 * c] = ldexpf(1.0f, -e);
    cs[2 * c + 1] = ldexpf(1.0f, e);
  }
}

// Z[p, c] = sum over splits (in split order) of the partials; written to Z
// (its own dtype and leading dimension) and/or to an FP64 copy z64 (ld = M).
// Loads are issued eight splits ahead of the (ordered) adds.
template <typename Acc, typename TZ>
__global__ __launch_bounds__(256) void k_reduce_splits(int M, int N, int nsplit,
                                                       const Acc *__restrict__ part,
                                                       TZ *__restrict__ Z, int64_t ldz,
                                                       double *__restrict__ z64) {
  // 64 outputs per workgroup, one per lane; wave w sums splits
  // [w q, (w + 1) q) of them in split order (q = ceil(nsplit / 4)), and the
  // four segment sums are added in segment order: a fixed order, with four
  // times the loads in flight of one lane walking all the splits
  __shared__ Acc seg[4][64];
  const int64_t MN = (int64_t)M * N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = (nsplit + 3) / 4;
  const int z0 = min(nsplit, w * q), z1 = min(nsplit, z0 + q);
  for (int64_t base = (int64_t)blockIdx.x * 64; base < MN; base += (int64_t)gridDim.x * 64) {
    const int64_t t = base + lane;
    Acc s = Acc(0);
    if (t < MN && z0 < z1) {
      s = part[t + (int64_t)z0 * MN];
      int z = z0 + 1;
      for (; z + 8 <= z1; z += 8) {
        Acc v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[t + (int64_t)(z + u) * MN];
#pragma unroll
        for (int u = 0; u < 8; ++u) s = s + v[u];
      }
      for (; z < z1; ++z) s = s + part[t + (int64_t)z * MN];
    }
    seg[w][lane] = s;
    __syncthreads();
    if (w == 0 && t < MN) {
      Acc r = seg[0][lane];
      for (int v = 1; v < 4; ++v)
        if (v * q < nsplit) r = r + seg[v][lane];
      const int64_t c = t / M, p = t - c * M;
      if (Z) Z[p + c * ldz] = (TZ)r;
      if (z64) z64[t] = (double)r;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ batched

// Persistent workgroups over the Gaussian-stage items of all problems (FP64
// and FP32 G): item = (problem, 64-row tile, 64-column tile, K split); each
// writes its partial block into the problem's partials area.
template <int DT>
__global__ __launch_bounds__(256) void k_batch_gemm(int count, const ms_problem *__restrict__ P,
                                                    const BatchEntry *__restrict__ E,
                                                    const BatchTotals *__restrict__ tot,
                                                    const unsigned char *__restrict__ yarea,
                                                    unsigned char *__restrict__ parea) {
  using F = Mf<DT>;
  const int64_t total = tot->gemm_items;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = batch_find_m<&BatchEntry::gemm_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    int64_t local = it - e.gemm_start;
    const int split = (int)(local % e.nsplit);
    local /= e.nsplit;
    const int tn = (int)(local % e.tiles_n);
    const int tm = (int)(local / e.tiles_n);
    const int M = (int)Q.k2, N = e.nc;
    const int64_t kb = (int64_t)split * e.kchunk, ke = min(Q.k, kb + e.kchunk);
    const auto *Y = reinterpret_cast<const typename F::TY *>(yarea + e.y_off);
    auto *Pz = reinterpret_cast<typename F::Acc *>(parea + e.part_off) + (int64_t)split * M * N;
    gemm_tile<DT>(M, N, static_cast<const typename F::TG *>(Q.G), Q.ldg, Y, Q.k, Pz, kb, ke, tm,
                  tn);
  }
}

// The 16-bit stage of a batch on the wide tiles: item = (problem, 256 x 144
// output tile, K split), one 256-thread workgroup per item at a time with
// the tile's two LDS stages.  The fast path is taken per problem (G aligned
// with a leading dimension a multiple of 8, k2 a multiple of 8, k a
// multiple of 32; Y, the batch's sketch area, is 256-byte aligned with
// leading dimension k).
static_assert(kBatchWideTM == kWTM && kBatchWideTN == kWTN, "batched wide tile shape");

template <int DT, int YT>
__global__ __launch_bounds__(kWThreads) void k_batch_gemm_wide(
    int count, const ms_problem *__restrict__ P, const BatchEntry *__restrict__ E,
    const BatchTotals *__restrict__ tot, const unsigned char *__restrict__ yarea,
    unsigned char *__restrict__ parea) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned short *lds = reinterpret_cast<unsigned short *>(smem_raw);
  const int64_t total = tot->gemm_items;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = batch_find_m<&BatchEntry::gemm_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    int64_t local = it - e.gemm_start;
    const int split = (int)(local % e.nsplit);
    local /= e.nsplit;
    const int tn = (int)(local % e.tiles_n);
    const int tm = (int)(local / e.tiles_n);
    const int M = (int)Q.k2, N = e.nc;
    const int64_t kb = (int64_t)split * e.kchunk, ke = min(Q.k, kb + e.kchunk);
    const float *Y = reinterpret_cast<const float *>(yarea + e.y_off);
    float *Pz = reinterpret_cast<float *>(parea + e.part_off) + (int64_t)split * M * N;
    const unsigned short *G = static_cast<const unsigned short *>(Q.G);
    const bool fast = (Q.ldg & 7) == 0 && ((uintptr_t)G & 15) == 0 && (M & 7) == 0 &&
                      (Q.k & 3) == 0 && ((uintptr_t)Y & 15) == 0 && (Q.k % kWKS) == 0 &&
                      (e.kchunk % kWKS) == 0;
    if (fast)
      gemm_tile_wide<DT, YT, true>(M, N, G, Q.ldg, Y, Q.k, nullptr, Pz, kb, ke, (int64_t)kWKS,
                                   tm * kWTM, tn * kWTN, lds);
    else
      gemm_tile_wide<DT, YT, false>(M, N, G, Q.ldg, Y, Q.k, nullptr, Pz, kb, ke, (int64_t)kWKS,
                                    tm * kWTM, tn * kWTN, lds);
    __syncthreads();  // the next item's first stage overwrites the LDS
  }
}

hipError_t launch_batch_gemm(int count, ms_dtype g_dtype, const ms_problem *P, const BatchEntry *E,
                             const BatchTotals *tot, const unsigned char *yarea,
                             unsigned char *parea, int grid, hipStream_t st, int yterms) {
  switch (g_dtype) {
    case MS_F64:
      hipLaunchKernelGGL(k_batch_gemm<DT_F64>, dim3(grid), dim3(256), 0, st, count, P, E, tot,
                         yarea, parea);
      break;
    case MS_F32:
      hipLaunchKernelGGL(k_batch_gemm<DT_F32>, dim3(grid), dim3(256), 0, st, count, P, E, tot,
                         yarea, parea);
      break;
    case MS_BF16:
      if (yterms == 3) {
        const hipError_t e =
            allow_dynamic_lds((const void *)k_batch_gemm_wide<DT_BF16, 3>, wide_lds_bytes<3>());
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_batch_gemm_wide<DT_BF16, 3>), dim3(grid), dim3(kWThreads),
                           wide_lds_bytes<3>(), st, count, P, E, tot, yarea, parea);
      } else {
        const hipError_t e =
            allow_dynamic_lds((const void *)k_batch_gemm_wide<DT_BF16, 1>, wide_lds_bytes<1>());
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_batch_gemm_wide<DT_BF16, 1>), dim3(grid), dim3(kWThreads),
                           wide_lds_bytes<1>(), st, count, P, E, tot, yarea, parea);
      }
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Z_p = sum over splits (in split order) of problem p's partials, as FP64.
template <typename Acc>
__global__ void k_batch_reduce(int count, const ms_problem *__restrict__ P,
                               const BatchEntry *__restrict__ E,
                               const unsigned char *__restrict__ parea,
                               unsigned char *__restrict__ zarea) {
  const int p = blockIdx.y;
  const BatchEntry &e = E[p];
  if (!e.valid) return;
  const int64_t MN = P[p].k2 * e.nc;
  const Acc *part = reinterpret_cast<const Acc *>(parea + e.part_off);
  double *Z = reinterpret_cast<double *>(zarea + e.z_off);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < MN;
       t += (int64_t)gridDim.x * blockDim.x) {
    Acc s = part[t];
    int z = 1;
    for (; z + 8 <= e.nsplit; z += 8) {
      Acc v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[t + (int64_t)(z + u) * MN];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = s + v[u];
    }
    for (; z < e.nsplit; ++z) s = s + part[t + (int64_t)z * MN];
    Z[t] = (double)s;
  }
}

hipError_t launch_batch_reduce(int count, ms_dtype g_dtype, const ms_problem *P,
                               const BatchEntry *E, const unsigned char *parea,
                               unsigned char *zarea, int max_mn, hipStream_t st) {
  const dim3 grid((unsigned)std::max(1, (max_mn + 255) / 256), (unsigned)count);
  if (g_dtype == MS_F64)
    hipLaunchKernelGGL(k_batch_reduce<double>, grid, dim3(256), 0, st, count, P, E, parea, zarea);
  else
    hipLaunchKernelGGL(k_batch_reduce<float>, grid, dim3(256), 0, st, count, P, E, parea, zarea);
  return hipGetLastError();
}

GemmPlan plan_gemm(int64_t M, int64_t N, int64_t K, ms_dtype g_dtype) {
  GemmPlan p{};
  p.M = (int)M;
  p.N = (int)N;
  p.K = K;
  const bool h16 = g_dtype == MS_BF16 || g_dtype == MS_F16;
  // 16-bit G: 256 x 144 tiles, about one workgroup per compute unit, at
  // least 512 K values per workgroup (so the partials stay small next to the
  // chunk of G and Y each workgroup reads); else 64 x 64 tiles, ~1024
  // workgroups, at least 128 K values each
  p.tiles_m = (int)(h16 ? (M + kWTM - 1) / kWTM : (M + 63) / 64);
  p.tiles_n = (int)(h16 ? (N + kWTN - 1) / kWTN : (N + 63) / 64);
  const int64_t ks = h16 ? kWKS : 4;
  const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
  const int64_t target = h16 ? 256 : 1024, kmin = h16 ? 512 : 128;
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>((target + tiles - 1) / tiles,
                                                      (K + kmin - 1) / kmin));
  ns = std::min<int64_t>(ns, 65535);
  int64_t kc = (K + ns - 1) / ns;
  kc = (kc + ks - 1) / ks * ks;
  if (kc < ks) kc = ks;
  p.kchunk = kc;
  p.nsplit = (int)((K + kc - 1) / kc);
  if (p.nsplit < 1) p.nsplit = 1;
  const size_t acc = g_dtype == MS_F64 ? 8 : 4;
  p.partial_bytes = (size_t)p.nsplit * (size_t)M * (size_t)N * acc;
  // FP16: the column scales follow the partials
  if (g_dtype == MS_F16) p.partial_bytes = align_up(p.partial_bytes) + (size_t)N * 2 * sizeof(float);
  p.ybf16_bytes = 0;
  return p;
}

// The wide 16-bit kernel over a plan's tiles and K splits (dynamic LDS:
// two stages of G's and Y's tiles).
template <int DT, int YT>
hipError_t launch_wide(const GemmPlan &p, const void *G, int64_t ldg, const void *Y, int64_t ldy,
                       void *partials, const float *cs, hipStream_t st) {
  const int xcds = dev_info().xcds;
  const int tiles = p.tiles_m * p.tiles_n;
  const dim3 grid((unsigned)((int64_t)xcds * tiles * ((p.nsplit + xcds - 1) / xcds)));
  constexpr int lds = wide_lds_bytes<YT>();
  const bool fast = (ldg & 7) == 0 && ((uintptr_t)G & 15) == 0 && (p.M & 7) == 0 &&
                    (ldy & 3) == 0 && ((uintptr_t)Y & 15) == 0 && (p.K % kWKS) == 0;
  const void *fn = fast ? (const void *)k_gemm_wide<DT, YT, true>
                        : (const void *)k_gemm_wide<DT, YT, false>;
  hipError_t e = allow_dynamic_lds(fn, lds);
  if (e != hipSuccess) return e;
  if (fast)
    hipLaunchKernelGGL((k_gemm_wide<DT, YT, true>), grid, dim3(kWThreads), lds, st, p.M, p.N,
                       p.K, static_cast<const unsigned short *>(G), ldg,
                       static_cast<const float *>(Y), ldy, static_cast<float *>(partials),
                       p.kchunk, p.tiles_m, tiles, p.nsplit, xcds, cs);
  else
    hipLaunchKernelGGL((k_gemm_wide<DT, YT, false>), grid, dim3(kWThreads), lds, st, p.M, p.N,
                       p.K, static_cast<const unsigned short *>(G), ldg,
                       static_cast<const float *>(Y), ldy, static_cast<float *>(partials),
                       p.kchunk, p.tiles_m, tiles, p.nsplit, xcds, cs);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmPlan &p, ms_dtype g_dtype, const void *G, int64_t ldg,
                       const void *Y, int64_t ldy, void *Z, int64_t ldz, double *z64,
                       void *partials, void *ybf16, hipStream_t st, int yterms) {
  (void)ybf16;
  if (p.M <= 0 || p.N <= 0) return hipSuccess;
  const int64_t MN = (int64_t)p.M * p.N;
  const unsigned rblocks = (unsigned)std::min<int64_t>((MN + 63) / 64, 65535);
  if (p.K <= 0) return hipErrorInvalidValue;
  const int xcds = dev_info().xcds;
  const int tiles = p.tiles_m * p.tiles_n;
  const dim3 grid((unsigned)((int64_t)xcds * tiles * ((p.nsplit + xcds - 1) / xcds)));
  const bool reduce = Z != nullptr || z64 != nullptr;  // otherwise the caller consumes the partials
  switch (g_dtype) {
    case MS_F64:
      hipLaunchKernelGGL(k_gemm_splitk<DT_F64>, grid, dim3(256), 0, st, p.M, p.N, p.K,
                         (const double *)G, ldg, (const double *)Y, ldy, (double *)partials,
                         p.kchunk, p.tiles_m, tiles, p.nsplit, xcds);
      if (reduce)
        hipLaunchKernelGGL((k_reduce_splits<double, double>), dim3(rblocks), dim3(256), 0, st, p.M,
                           p.N, p.nsplit, (const double *)partials, (double *)Z, ldz, z64);
      break;
    case MS_F32:
      hipLaunchKernelGGL(k_gemm_splitk<DT_F32>, grid, dim3(256), 0, st, p.M, p.N, p.K,
                         (const float *)G, ldg, (const float *)Y, ldy, (float *)partials,
                         p.kchunk, p.tiles_m, tiles, p.nsplit, xcds);
      if (reduce)
        hipLaunchKernelGGL((k_reduce_splits<float, float>), dim3(rblocks), dim3(256), 0, st, p.M,
                           p.N, p.nsplit, (const float *)partials, (float *)Z, ldz, z64);
      break;
    case MS_BF16: {
      const hipError_t e = yterms == 3
                               ? launch_wide<DT_BF16, 3>(p, G, ldg, Y, ldy, partials, nullptr, st)
                               : launch_wide<DT_BF16, 1>(p, G, ldg, Y, ldy, partials, nullptr, st);
      if (e != hipSuccess) return e;
      if (reduce)
        hipLaunchKernelGGL((k_reduce_splits<float, float>), dim3(rblocks), dim3(256), 0, st, p.M,
                           p.N, p.nsplit, (const float *)partials, (float *)Z, ldz, z64);
      break;
    }
    case MS_F16: {
      float *cs = reinterpret_cast<float *>(static_cast<unsigned char *>(partials) +
                                            align_up((size_t)p.nsplit * MN * sizeof(float)));
      hipLaunchKernelGGL(k_f16_col_scale, dim3((unsigned)p.N), dim3(256), 0, st, p.K,
                         (const float *)Y, ldy, cs);
      const hipError_t e = yterms == 3
                               ? launch_wide<DT_F16, 3>(p, G, ldg, Y, ldy, partials, cs, st)
                               : launch_wide<DT_F16, 1>(p, G, ldg, Y, ldy, partials, cs, st);
      if (e != hipSuccess) return e;
      if (reduce)
        hipLaunchKernelGGL((k_reduce_splits<float, float>), dim3(rblocks), dim3(256), 0, st, p.M,
                           p.N, p.nsplit, (const float *)partials, (float *)Z, ldz, z64);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ FP64-accumulating GEMV
// Z64 (M x N, ld M) = G Y64 for a narrow FP64 right operand (N <= 8), G of
// any stored dtype, all products and sums in FP64.  Used by the refinement
// correction, where the sketched residual must keep FP64 accuracy.  Thread p
// owns row p of Z; workgroup z takes a K chunk; partials are reduced in order.
template <typename TG>
__device__ __forceinline__ double g_as_f64(TG v);
template <>
__device__ __forceinline__ double g_as_f64<double>(double v) { return v; }
template <>
__device__ __forceinline__ double g_as_f64<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double g_as_f64<unsigned short>(unsigned short v) {
  return (double)__uint_as_float((uint32_t)v << 16);
}
template <>
__device__ __forceinline__ double g_as_f64<_Float16>(_Float16 v) { return (double)v; }

template <typename TG>
__device__ __forceinline__ void g_rows4(const TG *g, bool vec, int nvalid, double v[4]) {
  if (vec) {
    typedef TG V __attribute__((ext_vector_type(4)));
    const V a = gload(reinterpret_cast<const V *>(g));
    v[0] = g_as_f64<TG>(a.x);
    v[1] = g_as_f64<TG>(a.y);
    v[2] = g_as_f64<TG>(a.z);
    v[3] = g_as_f64<TG>(a.w);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = q < nvalid ? g_as_f64<TG>(gload(g + q)) : 0.0;
  }
}

// buf[m * 8 + c] = Y[m + c * ldy] for m < len, c < N (a chunk of a narrow
// FP64 right operand), eight loads per thread issued before their LDS
// stores (indices past the end read the last element and are not stored).
__device__ __forceinline__ void stage_rhs(const double *__restrict__ Y, int64_t ldy, int len,
                                          int N, double *buf) {
  constexpr int U = 8;
  const int total = len * N, bd = (int)blockDim.x;
  for (int t0 = threadIdx.x; t0 < total; t0 += U * bd) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = min(t0 + u * bd, total - 1);
      const int c = t / len, m = t - c * len;
      v[u] = Y[m + (int64_t)c * ldy];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * bd;
      if (t < total) {
        const int c = t / len, m = t - c * len;
        buf[m * 8 + c] = v[u];
      }
    }
  }
}

// The columns m = slot, slot + S, ... < len of a staged chunk: acc[q][c] +=
// G[row q, m] * buf[m * RH + c].  VEC (four aligned rows in range): eight
// columns' raw 4-row loads are issued before their products, with no
// condition around them (a column past len reads column len - 1 and is not
// used) and the conversion to FP64 at the use, so each lane keeps eight
// loads in flight instead of one.  Else one column at a time, row by row.
template <typename TG, int RH, bool VEC>
__device__ __forceinline__ void gemv_cols(const TG *__restrict__ g0, int64_t ldg, int nvalid,
                                          const double *buf, int slot, int S, int len, int N,
                                          double (&acc)[4][RH]) {
  if constexpr (VEC) {
    constexpr int U = 8;
    typedef TG V __attribute__((ext_vector_type(4)));
    for (int m = slot; m < len; m += U * S) {
      V raw[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        raw[u] = gload(reinterpret_cast<const V *>(g0 + (int64_t)min(m + u * S, len - 1) * ldg));
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int mm = m + u * S;
        if (mm < len) {
#pragma unroll
          for (int c = 0; c < RH; ++c)
            if (c < N) {
              const double y = buf[mm * RH + c];
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[q][c] += g_as_f64<TG>(raw[u][q]) * y;
            }
        }
      }
    }
  } else {
    for (int m = slot; m < len; m += S) {
      double g[4];
      g_rows4<TG>(g0 + (int64_t)m * ldg, false, nvalid, g);
#pragma unroll
      for (int c = 0; c < RH; ++c)
        if (c < N) {
          const double y = buf[m * RH + c];
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q][c] += g[q] * y;
        }
    }
  }
}

// Split-K partials of G Y in FP64 for narrow Y (N <= 8 columns; G's values
// promoted exactly): block (row tile of 256 rows, K split).  Each thread owns
// four rows; the block's threads form 256 / L slots (L threads per column of
// the tile) that take the split's columns round-robin, Y's rows staged in LDS
// 1024 at a time; the slots' sums are added in slot order.
template <typename TG>
__global__ __launch_bounds__(256) void k_gemv64_splitk(int M, int N, int64_t K,
                                                       const TG *__restrict__ G, int64_t ldg,
                                                       const double *__restrict__ Y, int64_t ldy,
                                                       double *__restrict__ part, int64_t kchunk) {
  constexpr int RH = 8, CH = 1024;  // stage_rhs stores with stride 8
  __shared__ double buf[CH * RH];
  const int mt0 = blockIdx.x * 256;
  const int rows = min(256, M - mt0);
  const int L = (rows + 3) / 4, S = (int)blockDim.x / L;
  const int rg = (int)threadIdx.x % L, slot = (int)threadIdx.x / L;
  const int row0 = mt0 + 4 * rg, nvalid = min(4, M - row0);
  const bool active = slot < S;
  const int64_t kb = (int64_t)blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  const bool vec = nvalid == 4 && (ldg & 3) == 0 && ((uintptr_t)G & (4 * sizeof(TG) - 1)) == 0;
  double acc[4][RH];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < RH; ++c) acc[q][c] = 0.0;
  for (int64_t c0 = kb; c0 < ke; c0 += CH) {
    const int len = (int)min((int64_t)CH, ke - c0);
    __syncthreads();
    stage_rhs(Y + c0, ldy, len, N, buf);
    __syncthreads();
    if (active) {
      if (vec)
        gemv_cols<TG, RH, true>(G + row0 + c0 * ldg, ldg, nvalid, buf, slot, S, len, N, acc);
      else
        gemv_cols<TG, RH, false>(G + row0 + c0 * ldg, ldg, nvalid, buf, slot, S, len, N, acc);
    }
  }
  __syncthreads();
  if (active)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < RH; ++c)
        if (c < N) buf[((int64_t)slot * 4 * L + 4 * rg + q) * RH + c] = acc[q][c];
  __syncthreads();
  double *P = part + (int64_t)blockIdx.y * M * N;
  for (int t = threadIdx.x; t < rows * N; t += blockDim.x) {
    const int c = t / rows, rr = t - c * rows;
    double s = buf[rr * RH + c];
    for (int z = 1; z < S; ++z) s += buf[((int64_t)z * 4 * L + rr) * RH + c];
    P[mt0 + rr + (int64_t)c * M] = s;
  }
}

// Refinement of a batch: partials of G Yr in FP64 (G's values promoted
// exactly), item = (problem, K split).  Each thread owns four rows of G; the
// 256 threads form 256 / L slots (L = ceil(k2 / 4) threads per column of G)
// that take the split's columns round-robin; Yr is staged in LDS 1024 rows at
// a time, and the slots' sums are added in slot order at the end.
template <typename TG>
__global__ __launch_bounds__(256) void k_batch_gemv(int count, const ms_problem *__restrict__ P,
                                                    const BatchEntry *__restrict__ E,
                                                    const BatchTotals *__restrict__ tot,
                                                    const unsigned char *__restrict__ yrarea,
                                                    unsigned char *__restrict__ gvarea) {
  constexpr int RH = kBatchMaxRefineRhs, CH = 1024;
  static_assert(RH == 8, "stage_rhs stores with stride 8");
  __shared__ double buf[CH * RH];
  const int64_t total = tot->gv_items;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = batch_find_m<&BatchEntry::gv_start>(E, count, it);
    const ms_problem &Q = P[p];
    const BatchEntry &e = E[p];
    if (!e.refine) continue;   // converged in an earlier step
    const int split = (int)(it - e.gv_start);
    const int M = (int)Q.k2, N = (int)Q.nrhs;
    const int L = (M + 3) / 4, S = (int)blockDim.x / L;
    const int rg = (int)threadIdx.x % L, slot = (int)threadIdx.x / L;
    const int row0 = 4 * rg, nvalid = min(4, M - row0);
    const bool active = slot < S;
    const int64_t kb = (int64_t)split * e.kchunk, ke = min(Q.k, kb + e.kchunk);
    const double *Yr = reinterpret_cast<const double *>(yrarea + e.yr_off);
    const TG *G = static_cast<const TG *>(Q.G);
    const bool vec = nvalid == 4 && (Q.ldg & 3) == 0 &&
                     ((uintptr_t)G & (4 * sizeof(TG) - 1)) == 0;
    double acc[4][RH];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < RH; ++c) acc[q][c] = 0.0;
    for (int64_t c0 = kb; c0 < ke; c0 += CH) {
      const int len = (int)min((int64_t)CH, ke - c0);
      __syncthreads();  // earlier readers of buf are done
      stage_rhs(Yr + c0, Q.k, len, N, buf);
      __syncthreads();
      if (active) {
        if (vec)
          gemv_cols<TG, RH, true>(G + row0 + c0 * Q.ldg, Q.ldg, nvalid, buf, slot, S, len, N,
                                  acc);
        else
          gemv_cols<TG, RH, false>(G + row0 + c0 * Q.ldg, Q.ldg, nvalid, buf, slot, S, len, N,
                                   acc);
      }
    }
    // slot sums in slot order: buf[(slot * 4L + row) * RH + c]
    __syncthreads();
    if (active)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < RH; ++c)
          if (c < N) buf[((int64_t)slot * 4 * L + row0 + q) * RH + c] = acc[q][c];
    __syncthreads();
    double *part = reinterpret_cast<double *>(gvarea + e.gv_off) + (int64_t)split * M * N;
    for (int t = threadIdx.x; t < M * N; t += blockDim.x) {
      const int c = t / M, row = t - c * M;
      double s = buf[row * RH + c];
      for (int z = 1; z < S; ++z) s += buf[((int64_t)z * 4 * L + row) * RH + c];
      part[row + (int64_t)c * M] = s;
    }
  }
}

hipError_t launch_batch_gemv(int count, ms_dtype g_dtype, const ms_problem *P,
                             const BatchEntry *E, const BatchTotals *tot,
                             const unsigned char *yrarea, unsigned char *gvarea, int grid,
                             hipStream_t st) {
  switch (g_dtype) {
    case MS_F64:
      hipLaunchKernelGGL(k_batch_gemv<double>, dim3(grid), dim3(256), 0, st, count, P, E, tot,
                         yrarea, gvarea);
      break;
    case MS_F32:
      hipLaunchKernelGGL(k_batch_gemv<float>, dim3(grid), dim3(256), 0, st, count, P, E, tot,
                         yrarea, gvarea);
      break;
    case MS_BF16:
      hipLaunchKernelGGL(k_batch_gemv<unsigned short>, dim3(grid), dim3(256), 0, st, count, P, E,
                         tot, yrarea, gvarea);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t gemv64_partial_bytes(int64_t M, int64_t N, int64_t K) {
  const int64_t ns = std::max<int64_t>(1, std::min<int64_t>(1024, (K + 511) / 512));
  return (size_t)ns * (size_t)M * (size_t)N * 8;
}

hipError_t launch_gemv64(int64_t M, int64_t N, int64_t K, ms_dtype g_dtype, const void *G,
                         int64_t ldg, const double *Y, int64_t ldy, double *z64, double *part,
                         hipStream_t st) {
  if (N > 8 || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(1024, (K + 511) / 512));
  const int64_t kc = (K + ns - 1) / ns;
  ns = (K + kc - 1) / kc;
  const dim3 grid((unsigned)((M + 255) / 256), (unsigned)ns);
  switch (g_dtype) {
    case MS_F64:
      hipLaunchKernelGGL(k_gemv64_splitk<double>, grid, dim3(256), 0, st, (int)M, (int)N, K,
                         (const double *)G, ldg, Y, ldy, part, kc);
      break;
    case MS_F32:
      hipLaunchKernelGGL(k_gemv64_splitk<float>, grid, dim3(256), 0, st, (int)M, (int)N, K,
                         (const float *)G, ldg, Y, ldy, part, kc);
      break;
    case MS_BF16:
      hipLaunchKernelGGL(k_gemv64_splitk<unsigned short>, grid, dim3(256), 0, st, (int)M, (int)N,
                         K, (const unsigned short *)G, ldg, Y, ldy, part, kc);
      break;
    case MS_F16:
      hipLaunchKernelGGL(k_gemv64_splitk<_Float16>, grid, dim3(256), 0, st, (int)M, (int)N, K,
                         (const _Float16 *)G, ldg, Y, ldy, part, kc);
      break;
    default:
      return hipErrorInvalidValue;
  }
  const int64_t MN = M * N;
  const unsigned rblocks = (unsigned)std::min<int64_t>((MN + 63) / 64, 65535);
  hipLaunchKernelGGL((k_reduce_splits<double, double>), dim3(rblocks), dim3(256), 0, st, (int)M,
                     (int)N, (int)ns, (const double *)part, (double *)nullptr, (int64_t)M, z64);
  return hipGetLastError();
}

}  // namespace ms
