// batched.hip -- many independent multisketch sketch-and-solve problems
// (Alg. 1 with S = G C, Higgins, Boman, Yamazaki, arXiv 2508.14209) solved
// together in six launches whose grids depend only on the device and on the
// workspace capacities, so the sequence can be captured in a HIP graph once
// and replayed with rewritten descriptors:
//
//   setup   one workgroup: per-problem plan (items, workspace offsets) by
//           block scans over the descriptors, status words cleared
//   zero    clear every problem's CountSketch accumulator
//   cs      persistent CountSketch over (problem, column tile, rows, buckets)
//   gemm    persistent Gaussian stage over (problem, row tile, column tile, K)
//   reduce  split-K partials summed in split order, per problem, into FP64 Z
//   qr      one workgroup per problem: Householder QR, Q^T Z_B, back solve
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

constexpr int kSetupThreads = 1024;

struct BatchCaps {
  int64_t y_bytes, part_bytes, z_bytes;
};

struct BatchLayout {
  size_t pstatus, entries, totals, yarea, parea, zarea, total;
};

BatchLayout batch_layout(int count, const BatchCaps &caps) {
  BatchLayout L;
  Carve cv;
  L.pstatus = cv.take((size_t)count * sizeof(int));
  L.entries = cv.take((size_t)count * sizeof(BatchEntry));
  L.totals = cv.take(sizeof(BatchTotals));
  L.yarea = cv.take((size_t)caps.y_bytes);
  L.parea = cv.take((size_t)caps.part_bytes);
  L.zarea = cv.take((size_t)caps.z_bytes);
  L.total = cv.off;
  return L;
}

__device__ __forceinline__ int64_t wave_excl_scan64(int64_t v, int64_t &wave_total) {
  const int lane = threadIdx.x & 63;
  int64_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  wave_total = __shfl(incl, 63, 64);
  return incl - v;
}

// Exclusive scan of v over the workgroup (1024 threads); returns the
// thread's offset and sets total.
__device__ int64_t block_excl_scan64(int64_t v, int64_t *sh, int64_t &total) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t wt;
  const int64_t ex = wave_excl_scan64(v, wt);
  if (lane == 0) sh[wave] = wt;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) off += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  total = tot;
  return off + ex;
}

__global__ __launch_bounds__(kSetupThreads) void k_batch_setup(
    int count, const ms_problem *__restrict__ P, int wdata, int accw, int64_t rows_item,
    int64_t kchunk, BatchCaps caps, BatchEntry *__restrict__ E, BatchTotals *__restrict__ tot,
    int *__restrict__ pstatus, int *status) {
  __shared__ int64_t sh[16];
  if (threadIdx.x == 0) *status = MS_OK;
  const int per = (count + (int)blockDim.x - 1) / (int)blockDim.x;
  const int p0 = min(count, (int)threadIdx.x * per), p1 = min(count, p0 + per);
  int64_t s_cs = 0, s_gm = 0, s_y = 0, s_pt = 0, s_z = 0, mx = 0;
  for (int p = p0; p < p1; ++p) {
    BatchEntry e;
    batch_entry(P[p], wdata, accw, rows_item, kchunk, e);
    s_cs += batch_cs_items(e);
    s_gm += batch_gemm_items(e);
    s_y += batch_y_bytes(P[p], e, wdata);
    s_pt += batch_part_bytes(P[p], e, accw);
    s_z += batch_z_bytes(P[p], e);
    if (e.valid) mx = max(mx, P[p].k2 * (int64_t)e.nc);
    pstatus[p] = e.valid ? MS_OK : MS_ERR_ARG;
  }
  __syncthreads();
  int64_t t_cs, t_gm, t_y, t_pt, t_z;
  int64_t o_cs = block_excl_scan64(s_cs, sh, t_cs);
  int64_t o_gm = block_excl_scan64(s_gm, sh, t_gm);
  int64_t o_y = block_excl_scan64(s_y, sh, t_y);
  int64_t o_pt = block_excl_scan64(s_pt, sh, t_pt);
  int64_t o_z = block_excl_scan64(s_z, sh, t_z);
  // the workspace areas were sized on the host; descriptors rewritten for a
  // graph replay must not need more
  const bool fits = t_y <= caps.y_bytes && t_pt <= caps.part_bytes && t_z <= caps.z_bytes;
  for (int p = p0; p < p1; ++p) {
    BatchEntry e;
    batch_entry(P[p], wdata, accw, rows_item, kchunk, e);
    if (!fits) e.valid = 0;
    e.cs_start = o_cs;
    e.gemm_start = o_gm;
    e.y_off = o_y;
    e.part_off = o_pt;
    e.z_off = o_z;
    o_cs += batch_cs_items(e);
    o_gm += batch_gemm_items(e);
    o_y += batch_y_bytes(P[p], e, wdata);
    o_pt += batch_part_bytes(P[p], e, accw);
    o_z += batch_z_bytes(P[p], e);
    E[p] = e;
    if (!e.valid) record_status(status, fits ? MS_ERR_ARG : MS_ERR_NOMEM);
    if (!fits) pstatus[p] = MS_ERR_NOMEM;
  }
  __shared__ int64_t mx_sh[16];
  int64_t m = mx;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (int64_t)__shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) mx_sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t mm = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mm = max(mm, mx_sh[w]);
    BatchTotals T{};
    T.cs_items = fits ? t_cs : 0;
    T.gemm_items = fits ? t_gm : 0;
    T.y_bytes = fits ? t_y : 0;
    T.part_bytes = t_pt;
    T.z_bytes = t_z;
    T.max_mn = mm;
    *tot = T;
  }
}

// Clear the accumulators of all problems (the first y_bytes of the area).
__global__ void k_batch_zero(const BatchTotals *__restrict__ tot, unsigned char *__restrict__ yarea) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  const int64_t n16 = tot->y_bytes / 16;
  u4 *y = reinterpret_cast<u4 *>(yarea);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n16;
       t += (int64_t)gridDim.x * blockDim.x)
    y[t] = u4{0u, 0u, 0u, 0u};
}

bool valid_dtypes(ms_dtype a, ms_dtype g) {
  return (a == MS_F64 && g == MS_F64) || (a == MS_F32 && (g == MS_F32 || g == MS_BF16));
}

int64_t rows_item_of(const ms_opts *o) {
  const int r = o ? o->batch_rows_log2 : 0;
  return (int64_t)1 << (r ? r : 15);
}
int64_t kchunk_of(const ms_opts *o) {
  const int r = o ? o->batch_kchunk_log2 : 0;
  return (int64_t)1 << (r ? r : 10);
}
bool valid_batch_opts(const ms_opts *o) {
  if (!o) return true;
  if (o->cs_mode != MS_CS_AUTO && o->cs_mode != MS_CS_LDS) return false;
  if (o->refine_steps != 0) return false;
  if (o->batch_rows_log2 != 0 && (o->batch_rows_log2 < 8 || o->batch_rows_log2 > 24)) return false;
  if (o->batch_kchunk_log2 != 0 && (o->batch_kchunk_log2 < 5 || o->batch_kchunk_log2 > 20))
    return false;
  return true;
}

// Host pass over the descriptors: validity, area sizes and launch maxima.
struct HostBatch {
  bool ok = true;
  BatchCaps caps{0, 0, 0};
  int max_k2 = 1, max_n = 1, max_nc = 2;
  int64_t max_mn = 1;
};

HostBatch host_batch(int count, const ms_problem *probs, ms_dtype a, ms_dtype g,
                     const ms_opts *o) {
  HostBatch H;
  const int wdata = (int)dtype_size(a);
  const int accw = g == MS_F64 ? 8 : 4;
  for (int p = 0; p < count; ++p) {
    BatchEntry e;
    batch_entry(probs[p], wdata, accw, rows_item_of(o), kchunk_of(o), e);
    if (!e.valid) {
      H.ok = false;
      return H;
    }
    H.caps.y_bytes += batch_y_bytes(probs[p], e, wdata);
    H.caps.part_bytes += batch_part_bytes(probs[p], e, accw);
    H.caps.z_bytes += batch_z_bytes(probs[p], e);
    H.max_k2 = std::max<int>(H.max_k2, (int)probs[p].k2);
    H.max_n = std::max<int>(H.max_n, (int)probs[p].n);
    H.max_nc = std::max<int>(H.max_nc, e.nc);
    H.max_mn = std::max<int64_t>(H.max_mn, probs[p].k2 * e.nc);
  }
  return H;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" {

size_t ms_batch_workspace_size(int count, const ms_problem *probs, ms_dtype a_dtype,
                               ms_dtype g_dtype, const ms_opts *opts) {
  if (count < 1 || count > 65535 || !probs || !valid_dtypes(a_dtype, g_dtype) ||
      !valid_batch_opts(opts))
    return 0;
  const HostBatch H = host_batch(count, probs, a_dtype, g_dtype, opts);
  if (!H.ok) return 0;
  return batch_layout(count, H.caps).total;
}

ms_status sketch_lstsq_batched(int count, const ms_problem *probs_host,
                               const ms_problem *probs_dev, ms_dtype a_dtype, ms_dtype g_dtype,
                               const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  if (count < 1 || count > 65535 || !probs_host || !probs_dev || !ws) return MS_ERR_ARG;
  if (!valid_dtypes(a_dtype, g_dtype)) return MS_ERR_ARG;
  if (opts && (opts->refine_steps != 0 || opts->cs_mode == MS_CS_SORTED ||
               opts->cs_mode == MS_CS_ATOMIC))
    return MS_ERR_UNSUPPORTED;
  if (!valid_batch_opts(opts)) return MS_ERR_ARG;
  const HostBatch H = host_batch(count, probs_host, a_dtype, g_dtype, opts);
  if (!H.ok) return MS_ERR_ARG;
  const BatchLayout L = batch_layout(count, H.caps);
  if (ws_bytes < L.total) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  unsigned char *base = static_cast<unsigned char *>(ws);
  int *status = reinterpret_cast<int *>(base);
  int *pstatus = reinterpret_cast<int *>(base + L.pstatus);
  BatchEntry *E = reinterpret_cast<BatchEntry *>(base + L.entries);
  BatchTotals *tot = reinterpret_cast<BatchTotals *>(base + L.totals);
  unsigned char *yarea = base + L.yarea, *parea = base + L.parea, *zarea = base + L.zarea;
  const DevInfo &di = dev_info();
  const int wdata = (int)dtype_size(a_dtype);
  const int accw = g_dtype == MS_F64 ? 8 : 4;

  hipLaunchKernelGGL(k_batch_setup, dim3(1), dim3(kSetupThreads), 0, st, count, probs_dev, wdata,
                     accw, rows_item_of(opts), kchunk_of(opts), H.caps, E, tot, pstatus, status);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    const int64_t n16 = H.caps.y_bytes / 16;
    const unsigned zb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n16 + 255) / 256, 8192));
    hipLaunchKernelGGL(k_batch_zero, dim3(zb), dim3(256), 0, st, tot, yarea);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int grid = di.cus;  // one 1024-thread workgroup per CU (128 KB of LDS each)
    e = a_dtype == MS_F64
            ? launch_batch_cs<double>(count, probs_dev, E, tot, yarea, pstatus, status, grid, st)
            : launch_batch_cs<float>(count, probs_dev, E, tot, yarea, pstatus, status, grid, st);
  }
  if (e == hipSuccess)
    e = launch_batch_gemm(count, g_dtype, probs_dev, E, tot, yarea, parea, di.cus * 4, st);
  if (e == hipSuccess)
    e = launch_batch_reduce(count, g_dtype, probs_dev, E, parea, zarea, (int)H.max_mn, st);
  if (e == hipSuccess)
    e = launch_batch_qr(count, H.max_k2, H.max_n, H.max_nc, probs_dev, E, zarea, pstatus, status,
                        st);
  return e == hipSuccess ? MS_OK : MS_ERR_DEVICE;
}

ms_status ms_batch_status(const void *ws, int count, int32_t *status_host, void *stream) {
  if (!ws || count < 1 || count > 65535 || !status_host) return MS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  Carve cv;
  const size_t o_p = cv.take((size_t)count * sizeof(int));
  int v = 0;
  if (hipMemcpyAsync(&v, ws, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MS_ERR_DEVICE;
  if (hipMemcpyAsync(status_host, static_cast<const unsigned char *>(ws) + o_p,
                     (size_t)count * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MS_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return MS_ERR_DEVICE;
  return (ms_status)v;
}

}  // extern "C"
