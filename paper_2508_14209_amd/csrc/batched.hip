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
//
// and, for each refinement step, five more: clear the residual sketches,
// residuals r = B - A X (FP64), their CountSketch, G (C r) in FP64 split-K
// partials, and one workgroup per problem that sums the partials and applies
// the kept Q and R to update X.
#include <algorithm>

#include "ms_internal.h"

namespace ms {

namespace {

constexpr int kSetupThreads = 1024;

struct BatchCaps {
  int64_t code_bytes;                         // packed bucket/sign words
  int64_t key_bytes;                          // sorted block keys (deterministic mode)
  int64_t y_bytes, part_bytes, z_bytes;       // first pass
  int64_t f_bytes, r_bytes, yr_bytes, gv_bytes;  // refinement (0 without)
};

struct BatchLayout {
  size_t pstatus, entries, totals, codearea, keyarea, yarea, parea, zarea, farea, rarea, yrarea,
      gvarea, total;
};

BatchLayout batch_layout(int count, const BatchCaps &caps) {
  BatchLayout L;
  Carve cv;
  L.pstatus = cv.take((size_t)count * sizeof(int));
  L.entries = cv.take((size_t)count * sizeof(BatchEntry));
  L.totals = cv.take(sizeof(BatchTotals));
  L.codearea = cv.take((size_t)caps.code_bytes);
  L.keyarea = cv.take((size_t)caps.key_bytes);
  L.yarea = cv.take((size_t)caps.y_bytes);
  L.parea = cv.take((size_t)caps.part_bytes);
  L.zarea = cv.take((size_t)caps.z_bytes);
  L.farea = cv.take((size_t)caps.f_bytes);
  L.rarea = cv.take((size_t)caps.r_bytes);
  L.yrarea = cv.take((size_t)caps.yr_bytes);
  L.gvarea = cv.take((size_t)caps.gv_bytes);
  L.total = cv.off;
  return L;
}

// The per-problem quantities the setup scans: work items of each persistent
// launch and bytes of each workspace area.
enum BatchQ { QCS, QGEMM, QRES, QRCS, QGV, QCODE, QY, QPART, QZ, QF, QR, QYR, QGVB,
              QBK, QBF, QBFR, QKEY, NQ };

__host__ __device__ inline void batch_quantities(const ms_problem &P, const BatchEntry &e,
                                                 int wdata, int accw, int64_t q[NQ]) {
  q[QCS] = batch_cs_items(e);
  q[QGEMM] = batch_gemm_items(e);
  q[QRES] = batch_res_items(P, e);
  q[QRCS] = batch_rcs_items(e);
  q[QGV] = batch_gv_items(e);
  q[QCODE] = batch_code_bytes(P, e);
  q[QY] = batch_y_bytes(P, e, wdata);
  q[QPART] = batch_part_bytes(P, e, accw);
  q[QZ] = batch_z_bytes(P, e);
  q[QF] = batch_f_bytes(P, e);
  q[QR] = batch_r_bytes(P, e);
  q[QYR] = batch_yr_bytes(P, e);
  q[QGVB] = batch_gv_bytes(P, e);
  q[QBK] = batch_bk_items(P, e);
  q[QBF] = batch_bf_items(e);
  q[QBFR] = batch_bfr_items(P, e);
  q[QKEY] = batch_key_bytes(P, e);
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
    int64_t kchunk, int refine, int det, int g16, BatchCaps caps, BatchEntry *__restrict__ E,
    BatchTotals *__restrict__ tot, int *__restrict__ pstatus, int *status) {
  __shared__ int64_t sh[16];
  if (threadIdx.x == 0) *status = MS_OK;
  const int per = (count + (int)blockDim.x - 1) / (int)blockDim.x;
  const int p0 = min(count, (int)threadIdx.x * per), p1 = min(count, p0 + per);
  int64_t sum[NQ] = {}, mx = 0;
  for (int p = p0; p < p1; ++p) {
    BatchEntry e;
    batch_entry(P[p], wdata, accw, rows_item, kchunk, refine, e, det, g16);
    int64_t q[NQ];
    batch_quantities(P[p], e, wdata, accw, q);
    for (int j = 0; j < NQ; ++j) sum[j] += q[j];
    if (e.valid) mx = max(mx, P[p].k2 * (int64_t)e.nc);
    pstatus[p] = e.valid ? MS_OK : MS_ERR_ARG;
  }
  __syncthreads();
  int64_t off[NQ], total[NQ];
  for (int j = 0; j < NQ; ++j) off[j] = block_excl_scan64(sum[j], sh, total[j]);
  // the workspace areas were sized on the host; descriptors rewritten for a
  // graph replay must not need more
  // packed bucket words only when the capacity's rows cover the batch's (a
  // replay with more rows reads h and s in every item instead)
  const bool codes = total[QCODE] <= caps.code_bytes;
  const bool fits = total[QY] <= caps.y_bytes && total[QPART] <= caps.part_bytes &&
                    total[QZ] <= caps.z_bytes && total[QF] <= caps.f_bytes &&
                    total[QR] <= caps.r_bytes && total[QYR] <= caps.yr_bytes &&
                    total[QGVB] <= caps.gv_bytes && total[QKEY] <= caps.key_bytes;
  for (int p = p0; p < p1; ++p) {
    BatchEntry e;
    batch_entry(P[p], wdata, accw, rows_item, kchunk, refine, e, det, g16);
    const bool valid = e.valid != 0;
    if (!fits) e.valid = 0;
    int64_t q[NQ];
    batch_quantities(P[p], e, wdata, accw, q);
    e.cs_start = off[QCS];
    e.gemm_start = off[QGEMM];
    e.res_start = off[QRES];
    e.rcs_start = off[QRCS];
    e.gv_start = off[QGV];
    e.code_off = codes && batch_packs(e) ? off[QCODE] : -1;
    e.y_off = off[QY];
    e.part_off = off[QPART];
    e.z_off = off[QZ];
    e.f_off = off[QF];
    e.r_off = off[QR];
    e.yr_off = off[QYR];
    e.gv_off = off[QGVB];
    e.bk_start = off[QBK];
    e.bf_start = off[QBF];
    e.bfr_start = off[QBFR];
    e.key_off = off[QKEY];
    for (int j = 0; j < NQ; ++j) off[j] += q[j];
    E[p] = e;
    if (!valid) record_status(status, MS_ERR_ARG);
    if (!fits) {
      record_status(status, MS_ERR_NOMEM);
      pstatus[p] = MS_ERR_NOMEM;
    }
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
    T.cs_items = fits ? total[QCS] : 0;
    T.gemm_items = fits ? total[QGEMM] : 0;
    T.res_items = fits ? total[QRES] : 0;
    T.rcs_items = fits ? total[QRCS] : 0;
    T.gv_items = fits ? total[QGV] : 0;
    T.bk_items = fits ? total[QBK] : 0;
    T.bf_items = fits ? total[QBF] : 0;
    T.bfr_items = fits ? total[QBFR] : 0;
    T.y_bytes = fits ? total[QY] : 0;
    T.yr_bytes = fits ? total[QYR] : 0;
    T.part_bytes = total[QPART];
    T.z_bytes = total[QZ];
    T.max_mn = mm;
    *tot = T;
  }
}

// Clear the CountSketch outputs (Y, or Yr for the residual sketches) that
// are accumulated with atomic adds: those of problems whose rows are split
// over several items.  A problem of one row segment has each slot of its
// output stored exactly once by the owner of its (column tile, bucket tile),
// so it needs no clearing.  Workgroup row y takes problems y, y + gridDim.y, ...
__global__ void k_batch_zero(int count, const ms_problem *__restrict__ P,
                             const BatchEntry *__restrict__ E, int residual, int wdata,
                             unsigned char *__restrict__ area) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  for (int p = blockIdx.y; p < count; p += gridDim.y) {
    const BatchEntry &e = E[p];
    if (!e.valid || e.nsegs <= 1) continue;
    const int64_t bytes = residual ? batch_yr_bytes(P[p], e) : batch_y_bytes(P[p], e, wdata);
    u4 *y = reinterpret_cast<u4 *>(area + (residual ? e.yr_off : e.y_off));
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < bytes / 16;
         t += (int64_t)gridDim.x * blockDim.x)
      y[t] = u4{0u, 0u, 0u, 0u};
  }
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
int refine_of(const ms_opts *o) { return o ? o->refine_steps : 0; }
int det_of(const ms_opts *o) { return (o && o->cs_mode == MS_CS_SORTED) ? 1 : 0; }
bool valid_batch_opts(const ms_opts *o) {
  if (!o) return true;
  if (o->cs_mode != MS_CS_AUTO && o->cs_mode != MS_CS_LDS && o->cs_mode != MS_CS_SORTED)
    return false;
  if (o->refine_steps < 0 || o->refine_steps > 64) return false;
  if (o->batch_rows_log2 != 0 && (o->batch_rows_log2 < 8 || o->batch_rows_log2 > 24)) return false;
  if (o->batch_kchunk_log2 != 0 && (o->batch_kchunk_log2 < 5 || o->batch_kchunk_log2 > 20))
    return false;
  if (!(o->gauss_y_terms == 0 || o->gauss_y_terms == 1 || o->gauss_y_terms == 3)) return false;
  if (o->refine_tol_log2 < 0 || o->refine_tol_log2 > 60) return false;
  return true;
}

// Host pass over the descriptors: validity, area sizes and launch maxima.
struct HostBatch {
  bool ok = true, refine_rhs_ok = true;
  BatchCaps caps{0, 0, 0, 0, 0, 0, 0, 0, 0};
  int max_k2 = 1, max_n = 1, max_nc = 2;
  int64_t max_mn = 1;
};

HostBatch host_batch(int count, const ms_problem *probs, ms_dtype a, ms_dtype g,
                     const ms_opts *o) {
  HostBatch H;
  const int wdata = (int)dtype_size(a);
  const int accw = g == MS_F64 ? 8 : 4;
  const int refine = refine_of(o) > 0;
  for (int p = 0; p < count; ++p) {
    if (refine && probs[p].nrhs > kBatchMaxRefineRhs) {
      H.refine_rhs_ok = false;
      return H;
    }
    BatchEntry e;
    batch_entry(probs[p], wdata, accw, rows_item_of(o), kchunk_of(o), refine, e, det_of(o),
                g == MS_BF16 ? 1 : 0);
    if (!e.valid) {
      H.ok = false;
      return H;
    }
    int64_t q[NQ];
    batch_quantities(probs[p], e, wdata, accw, q);
    H.caps.code_bytes += q[QCODE];
    H.caps.key_bytes += q[QKEY];
    H.caps.y_bytes += q[QY];
    H.caps.part_bytes += q[QPART];
    H.caps.z_bytes += q[QZ];
    H.caps.f_bytes += q[QF];
    H.caps.r_bytes += q[QR];
    H.caps.yr_bytes += q[QYR];
    H.caps.gv_bytes += q[QGVB];
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
  if (!H.ok || !H.refine_rhs_ok) return 0;
  return batch_layout(count, H.caps).total;
}

ms_status sketch_lstsq_batched(int count, const ms_problem *probs_host,
                               const ms_problem *probs_dev, ms_dtype a_dtype, ms_dtype g_dtype,
                               const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  if (count < 1 || count > 65535 || !probs_host || !probs_dev || !ws) return MS_ERR_ARG;
  if (a_dtype == MS_F32 && g_dtype == MS_F16) return MS_ERR_UNSUPPORTED;
  if (!valid_dtypes(a_dtype, g_dtype)) return MS_ERR_ARG;
  if (opts && opts->cs_mode == MS_CS_ATOMIC) return MS_ERR_UNSUPPORTED;
  if (!valid_batch_opts(opts)) return MS_ERR_ARG;
  const HostBatch H = host_batch(count, probs_host, a_dtype, g_dtype, opts);
  if (!H.refine_rhs_ok) return MS_ERR_UNSUPPORTED;
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
  unsigned char *codearea = base + L.codearea, *keyarea = base + L.keyarea;
  unsigned char *farea = base + L.farea, *rarea = base + L.rarea, *yrarea = base + L.yrarea,
                *gvarea = base + L.gvarea;
  const DevInfo &di = dev_info();
  const int wdata = (int)dtype_size(a_dtype);
  const int accw = g_dtype == MS_F64 ? 8 : 4;
  const int refine = refine_of(opts);
  const int det = det_of(opts);

  hipLaunchKernelGGL(k_batch_setup, dim3(1), dim3(kSetupThreads), 0, st, count, probs_dev, wdata,
                     accw, rows_item_of(opts), kchunk_of(opts), refine > 0 ? 1 : 0, det,
                     g_dtype == MS_BF16 ? 1 : 0, H.caps,
                     E, tot, pstatus, status);
  hipError_t e = hipGetLastError();
  auto zero = [&](int residual, unsigned char *area) {
    hipLaunchKernelGGL(k_batch_zero, dim3(32, (unsigned)std::min(count, 2048)), dim3(256), 0, st,
                       count, probs_dev, E, residual, wdata, area);
    return hipGetLastError();
  };
  if (det) {
    // deterministic: sorted block keys, then the block-ordered fold of every
    // column (each output slot stored once, no clearing)
    if (e == hipSuccess)
      e = launch_batch_bf_keys(count, probs_dev, E, tot, keyarea, pstatus, status, di.cus * 4, st);
    if (e == hipSuccess)
      e = a_dtype == MS_F64
              ? launch_batch_bf_fold<double, 0>(count, probs_dev, E, tot, keyarea, nullptr, yarea,
                                                di.cus, st)
              : launch_batch_bf_fold<float, 0>(count, probs_dev, E, tot, keyarea, nullptr, yarea,
                                               di.cus, st);
  }
  if (e == hipSuccess && !det) e = zero(0, yarea);
  if (e == hipSuccess && !det)
    e = launch_batch_pack(count, probs_dev, E, codearea, pstatus, status, st);
  if (e == hipSuccess && !det) {
    const int grid = di.cus;  // one 1024-thread workgroup per CU (128 KB of LDS each)
    e = a_dtype == MS_F64
            ? launch_batch_cs<double>(count, probs_dev, E, tot, codearea, yarea, pstatus, status,
                                      grid, st)
            : launch_batch_cs<float>(count, probs_dev, E, tot, codearea, yarea, pstatus, status,
                                     grid, st);
  }
  if (e == hipSuccess)
    e = launch_batch_gemm(count, g_dtype, probs_dev, E, tot, yarea, parea,
                          g_dtype == MS_BF16 ? di.cus : di.cus * 4, st,
                          (opts && opts->gauss_y_terms == 1) ? 1 : 3);
  if (e == hipSuccess)
    e = launch_batch_reduce(count, g_dtype, probs_dev, E, parea, zarea, (int)H.max_mn, st);
  if (e == hipSuccess)
    e = launch_batch_qr(count, H.max_k2, H.max_n, H.max_nc, probs_dev, E, zarea, farea, pstatus,
                        status, st, det);
  // refinement: r = B - A X (FP64); X += R^{-1} Q^T G (C r)
  for (int it = 0; it < refine && e == hipSuccess; ++it) {
    if (!det) e = zero(1, yrarea);
    if (e == hipSuccess)
      e = a_dtype == MS_F64
              ? launch_batch_residual<double>(count, probs_dev, E, tot, rarea, di.cus * 8, st)
              : launch_batch_residual<float>(count, probs_dev, E, tot, rarea, di.cus * 8, st);
    if (e == hipSuccess)
      e = det ? launch_batch_bf_fold<double, 1>(count, probs_dev, E, tot, keyarea, rarea, yrarea,
                                                di.cus, st)
              : launch_batch_cs_res(count, probs_dev, E, tot, codearea, rarea, yrarea, pstatus,
                                    status, di.cus, st);
    if (e == hipSuccess)
      e = launch_batch_gemv(count, g_dtype, probs_dev, E, tot, yrarea, gvarea, di.cus * 4, st);
    if (e == hipSuccess)
      e = launch_batch_apply_solve(count, probs_dev, E, gvarea, farea, pstatus, status, st,
                                   opts ? opts->refine_tol_log2 : 0);
  }
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
