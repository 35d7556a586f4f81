// gen.hip -- seeded synthetic least-squares requests generated on the device
// (the serving workload: matrices of a prescribed condition number, as in the
// experiments of Sec. 6.3, arriving faster than a host could upload them).
//
//   A = Z diag(D) Q   (d x n FP32): Z with independent N(0,1) entries,
//                     D_j = kappa^(-j/(n-1)), Q = H(u1) H(u2) with
//                     H(u) = I - 2 u u^T and unit Gaussian directions u1, u2
//                     (orthogonal; mixes every column into every other);
//   x* (n x nrhs) N(0,1);  B = A x* + noise N(0,1) (FP32);
//   h uniform in [0, k), s uniform in {-1, +1};
//   G (k2 x k) = N(0,1) / sqrt(k2) drawn in FP32 (stored FP32, BF16 rounded
//   to nearest even, or FP64 exactly).
//
// Normal variates are Box-Muller pairs of uniforms cut from counter-based
// 64-bit words: word c of a stream is SplitMix64's (c+1)-th output from that
// stream's state (Steele, Lea and Flood, OOPSLA 2014), the stream states
// being SplitMix64-finalised (seed, stream tag).  Every value is a function
// of (seed, its position), so a request is the same on any device, stream or
// launch shape.  The logarithm, square root, sine and cosine are the
// hardware approximations (inputs in revolutions for the circular ones):
// synthetic data, not part of the method.
//
// One thread per row of A: the row of Z diag(D) is formed in registers, its
// inner products with u1 and u2 give the row of A,
//   a H(u1) H(u2) = a - 2 t1 u1 - 2 (t2 - 2 t1 c) u2,  t1 = a.u1, t2 = a.u2,
//   c = u1.u2,
// which is written once (coalesced over the wave's rows) and multiplied by
// x* for B.  One pass of writes over A and B; nothing is read back.
#include <algorithm>
#include <cmath>

#include "ms_internal.h"

namespace ms {

namespace {

constexpr int kGenMaxN = 128, kGenMaxR = 8;
constexpr int64_t kGenMax31 = 0x7ffffffe;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
enum : uint64_t { kStreamZ = 1, kStreamU = 2, kStreamX = 3, kStreamNoise = 4, kStreamHS = 5,
                  kStreamG = 6 };

__host__ __device__ __forceinline__ uint64_t sm_final(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return sm_final(seed + tag * kGamma);
}

__device__ __forceinline__ uint64_t word(uint64_t key, uint64_t c) {
  return sm_final(key + (c + 1) * kGamma);
}

// Two independent N(0,1) values from one 64-bit word: u1 in (0, 1] from the
// high half, u2 in [0, 1) from the low half; r = sqrt(-2 ln u1).
__device__ __forceinline__ float2 normal2(uint64_t w) {
  const float inv32 = 2.3283064365386963e-10f;  // 2^-32
  const float u1 = ((float)(uint32_t)(w >> 32) + 1.0f) * inv32;
  const float u2 = (float)(uint32_t)w * inv32;
  // -2 ln u1 = -2 ln(2) log2(u1)
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  return make_float2(r * __builtin_amdgcn_cosf(u2), r * __builtin_amdgcn_sinf(u2));
}

struct GenArgs {
  int64_t d, k;
  int n, nrhs;
  double log10_kappa;
  float noise;
  uint64_t seed;
  float *A;
  int64_t lda;
  float *B;
  int64_t ldb;
  float *xstar;
  int32_t *h;
  int8_t *s;
};

__global__ __launch_bounds__(256) void k_gen_rows(GenArgs g) {
  __shared__ float sD[kGenMaxN], sU1[kGenMaxN], sU2[kGenMaxN];
  __shared__ float sX[kGenMaxN * kGenMaxR];
  __shared__ float red[2][3];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = g.n, nrhs = g.nrhs;
  // per block: D, the normalised reflector directions and x*
  float u1 = 0.0f, u2 = 0.0f;
  if (tid < kGenMaxN) {
    if (tid < n) {
      const float2 z = normal2(word(stream_key(g.seed, kStreamU), (uint64_t)tid));
      u1 = z.x;
      u2 = z.y;
      sD[tid] = n > 1 ? (float)pow(10.0, -g.log10_kappa * (double)tid / (double)(n - 1)) : 1.0f;
    } else {
      sD[tid] = 0.0f;
    }
    float q11 = u1 * u1, q22 = u2 * u2, q12 = u1 * u2;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      q11 += __shfl_xor(q11, o, 64);
      q22 += __shfl_xor(q22, o, 64);
      q12 += __shfl_xor(q12, o, 64);
    }
    if (lane == 0) {
      red[wave][0] = q11;
      red[wave][1] = q22;
      red[wave][2] = q12;
    }
  }
  const uint64_t kx = stream_key(g.seed, kStreamX);
  for (int e = tid; e < n * nrhs; e += blockDim.x) {
    const float2 z = normal2(word(kx, (uint64_t)(e >> 1)));
    sX[e] = (e & 1) ? z.y : z.x;
  }
  __syncthreads();
  const float n11 = red[0][0] + red[1][0], n22 = red[0][1] + red[1][1];
  const float i1 = n11 > 0.0f ? 1.0f / sqrtf(n11) : 0.0f;
  const float i2 = n22 > 0.0f ? 1.0f / sqrtf(n22) : 0.0f;
  const float c = (red[0][2] + red[1][2]) * i1 * i2;
  if (tid < kGenMaxN) {
    sU1[tid] = u1 * i1;
    sU2[tid] = u2 * i2;
  }
  __syncthreads();
  if (blockIdx.x == 0 && g.xstar)
    for (int e = tid; e < n * nrhs; e += blockDim.x) g.xstar[e] = sX[e];

  const uint64_t kz = stream_key(g.seed, kStreamZ), kn = stream_key(g.seed, kStreamNoise),
                 khs = stream_key(g.seed, kStreamHS);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < g.d;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (g.h) {
      const uint64_t w = word(khs, (uint64_t)i);
      g.h[i] = (int32_t)(((w >> 32) * (uint64_t)g.k) >> 32);
      g.s[i] = (w & 1u) ? (int8_t)-1 : (int8_t)1;
    }
    if (!g.A) continue;
    float a[kGenMaxN];
    float t1 = 0.0f, t2 = 0.0f;
#pragma unroll
    for (int p = 0; p < kGenMaxN / 2; ++p) {
      if (2 * p < n) {
        const float2 z = normal2(word(kz, (uint64_t)i * (kGenMaxN / 2) + p));
        a[2 * p] = z.x * sD[2 * p];
        a[2 * p + 1] = z.y * sD[2 * p + 1];
        t1 += a[2 * p] * sU1[2 * p] + a[2 * p + 1] * sU1[2 * p + 1];
        t2 += a[2 * p] * sU2[2 * p] + a[2 * p + 1] * sU2[2 * p + 1];
      }
    }
    const float f1 = 2.0f * t1, f2 = 2.0f * (t2 - 2.0f * t1 * c);
    float b[kGenMaxR];
#pragma unroll
    for (int r = 0; r < kGenMaxR; ++r) b[r] = 0.0f;
#pragma unroll
    for (int j = 0; j < kGenMaxN; ++j) {
      if (j < n) {
        const float v = a[j] - f1 * sU1[j] - f2 * sU2[j];
        g.A[i + (int64_t)j * g.lda] = v;
#pragma unroll
        for (int r = 0; r < kGenMaxR; ++r)
          if (r < nrhs) b[r] += v * sX[j + r * n];
      }
    }
    if (!g.B) continue;
#pragma unroll
    for (int q = 0; q < kGenMaxR / 2; ++q) {
      if (2 * q < nrhs) {
        const float2 z = normal2(word(kn, (uint64_t)i * (kGenMaxR / 2) + q));
        g.B[i + (int64_t)(2 * q) * g.ldb] = b[2 * q] + g.noise * z.x;
        if (2 * q + 1 < nrhs) g.B[i + (int64_t)(2 * q + 1) * g.ldb] = b[2 * q + 1] + g.noise * z.y;
      }
    }
  }
}

// FP32 -> BF16 bits, nearest even (finite values; G holds no NaN).
__device__ __forceinline__ unsigned short gen_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// G's entries e = 8 t .. 8 t + 7 (linear, column-major k2 x k with ld k2).
__global__ __launch_bounds__(256) void k_gen_gauss(int64_t count, uint64_t key, float scale,
                                                   int dt, void *G) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t * 8 < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float2 z = normal2(word(key, (uint64_t)(4 * t + q)));
      v[2 * q] = z.x * scale;
      v[2 * q + 1] = z.y * scale;
    }
    const int64_t e0 = 8 * t;
    const int m = count - e0 < 8 ? (int)(count - e0) : 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < m) {
        if (dt == MS_F32) static_cast<float *>(G)[e0 + q] = v[q];
        else if (dt == MS_BF16) static_cast<unsigned short *>(G)[e0 + q] = gen_bf16(v[q]);
        else static_cast<double *>(G)[e0 + q] = (double)v[q];
      }
    }
  }
}

}  // namespace

}  // namespace ms

using namespace ms;

extern "C" ms_status ms_gen_lstsq_request(uint64_t seed, int64_t d, int64_t n, int64_t nrhs,
                                          double kappa, double noise, int64_t k, int64_t k2,
                                          ms_dtype g_dtype, float *A, int64_t lda, float *B,
                                          int64_t ldb, float *xstar, int32_t *h, int8_t *s,
                                          void *G, void *stream) {
  if (d < 1 || n < 1 || n > kGenMaxN || nrhs < 1 || nrhs > kGenMaxR || k < 1 || k > kGenMax31 ||
      k2 < 1 || k2 > kGenMax31)
    return MS_ERR_ARG;
  if (!(kappa >= 1.0) || !std::isfinite(kappa) || !std::isfinite(noise)) return MS_ERR_ARG;
  if ((A && lda < d) || (B && (ldb < d || !A)) || ((h != nullptr) != (s != nullptr)))
    return MS_ERR_ARG;
  if (G && g_dtype != MS_F32 && g_dtype != MS_BF16 && g_dtype != MS_F64) return MS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (A || B || xstar || h) {
    GenArgs g{d, k, (int)n, (int)nrhs, std::log10(kappa), (float)noise, seed, A, lda, B, ldb,
              xstar, h, s};
    const unsigned blocks = (unsigned)std::min<int64_t>((d + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gen_rows, dim3(blocks), dim3(256), 0, st, g);
    if (hipGetLastError() != hipSuccess) return MS_ERR_DEVICE;
  }
  if (G) {
    const int64_t count = k2 * k;
    const unsigned blocks = (unsigned)std::min<int64_t>((count + 2047) / 2048, 8192);
    hipLaunchKernelGGL(k_gen_gauss, dim3(blocks), dim3(256), 0, st, count,
                       stream_key(seed, kStreamG), (float)(1.0 / std::sqrt((double)k2)),
                       (int)g_dtype, G);
    if (hipGetLastError() != hipSuccess) return MS_ERR_DEVICE;
  }
  return MS_OK;
}
