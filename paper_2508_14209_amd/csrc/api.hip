// api.hip -- the C ABI of libmsketch (include/msketch.h): argument checks,
// workspace layout and the order of launches for each entry point.  Every
// step of the path runs in this library's kernels; this file only validates,
// carves the caller's workspace and enqueues.
#include <mutex>

#include "ms_internal.h"

namespace ms {

// ------------------------------------------------------------------ device info
namespace {
std::mutex g_mu;
constexpr int kMaxDev = 64;
DevInfo g_info[kMaxDev];
bool g_have[kMaxDev];
struct LdsKey {
  const void *fn;
  int dev;
  int bytes;
};
LdsKey g_lds[256];
int g_nlds = 0;
}  // namespace

const DevInfo &dev_info() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) dev = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_have[dev]) {
    DevInfo d;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) d.cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      d.lds_per_block = v;
    if (d.cus <= 0) d.cus = 256;
    if (d.lds_per_block <= 0) d.lds_per_block = 65536;
    g_info[dev] = d;
    g_have[dev] = true;
  }
  return g_info[dev];
}

hipError_t allow_dynamic_lds(const void *kernel, int bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (int i = 0; i < g_nlds; ++i)
      if (g_lds[i].fn == kernel && g_lds[i].dev == dev && g_lds[i].bytes >= bytes) return hipSuccess;
  }
  if (bytes <= 65536) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_nlds < 256) g_lds[g_nlds++] = LdsKey{kernel, dev, bytes};
  return hipSuccess;
}

// refine.hip
hipError_t launch_residual_f32(int64_t d, int64_t n, int64_t nrhs, const float *A, int64_t lda,
                               const float *B, int64_t ldb, const double *X, int64_t ldx,
                               double *r, int64_t ldr, hipStream_t st);
hipError_t launch_residual_f64(int64_t d, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                               const double *B, int64_t ldb, const double *X, int64_t ldx,
                               double *r, int64_t ldr, hipStream_t st);
hipError_t launch_axpy_update(int64_t n, int64_t nrhs, const double *dX, double *X, int64_t ldx,
                              hipStream_t st);

// ------------------------------------------------------------------ layouts

namespace {

constexpr int64_t kMax31 = 0x7ffffffe;

int resolve_mode(const ms_opts *o) {
  const int m = o ? o->cs_mode : MS_CS_AUTO;
  return m == MS_CS_AUTO ? MS_CS_LDS : m;
}

struct CsLayout {
  size_t code = 0, cnt = 0, off = 0, cursor = 0, sperm = 0, tab = 0, tab_bytes = 0;
  size_t bkeys = 0, bkeys_bytes = 0;  // the block fold's sorted keys (sorted mode)
  size_t part = 0, part_bytes = 0;
  size_t tplan = 0, tplan_bytes = 0;  // the tiled CountSketch's plan (k > 16384)
};

// ncols, wd: columns and element bytes of the sketched operand (the LDS
// variant's per-die partial buffer, when its schedule pays for the shape).
void carve_cs(Carve &cv, CsLayout &L, int64_t d, int64_t k, int mode, int64_t ncols, int64_t wd) {
  if (mode == MS_CS_SORTED && cs_blockfold_supported(d, k, 1, 8)) {
    // the block fold (FP64 sizing, so that the FP64 residual's sketch fits too)
    L.bkeys_bytes = cs_blockfold_key_bytes(d);
    L.bkeys = cv.take(L.bkeys_bytes);
  } else if (mode == MS_CS_SORTED) {
    L.cnt = cv.take((size_t)k * 4);
    L.off = cv.take((size_t)(k + 1) * 4);
    L.cursor = cv.take((size_t)k * 4);
    L.sperm = cv.take((size_t)d * 4);
    // the blocked plan's count table (k <= 16384)
    L.tab_bytes = plan_blocked_bytes(d, k);
    if (L.tab_bytes) L.tab = cv.take(L.tab_bytes);
  } else {
    // the tiled CountSketch's plan comes first, right after the status block
    if (mode == MS_CS_LDS) {
      L.tplan_bytes = cs_tile_plan_bytes(d, k);
      if (L.tplan_bytes) L.tplan = cv.take(L.tplan_bytes);
    }
    L.code = cv.take((size_t)d * 4);
    if (mode == MS_CS_LDS && !L.tplan_bytes) {
      L.part_bytes = cs_part_bytes(d, k, ncols, wd);
      if (L.part_bytes) L.part = cv.take(L.part_bytes);
    }
  }
}

// The LDS CountSketch of this call runs as the tiled CountSketch: the plan
// has room in the workspace, the device can run it, and no schedule
// override of the single-tile kernels was asked for.
bool use_tiled(const CsLayout &L, int64_t d, int64_t k, const CsTuning &tune) {
  return L.tplan_bytes && !tune.grid_variant && !tune.cols_per_wg && cs_tiled_supported(d, k);
}

struct LstsqLayout {
  CsLayout cs;
  size_t y = 0, partials = 0, z64 = 0, qr = 0, fact = 0, tau = 0;
  size_t r = 0, yr = 0, zr = 0, gv = 0, dx = 0;
  size_t total = 0;
};

LstsqLayout lstsq_layout(int64_t d, int64_t n, int64_t nrhs, int64_t k, int64_t k2,
                         ms_dtype a_dtype, ms_dtype g_dtype, int mode, int refine) {
  LstsqLayout L;
  Carve cv;
  const int64_t nc = n + nrhs;
  carve_cs(cv, L.cs, d, k, mode, nc, dtype_size(a_dtype));
  L.y = cv.take((size_t)k * nc * dtype_size(a_dtype));
  L.partials = cv.take(plan_gemm(k2, nc, k, g_dtype).partial_bytes);
  L.z64 = cv.take((size_t)k2 * nc * 8);
  L.qr = cv.take(qr_workspace_bytes(k2, n, nrhs));
  L.fact = cv.take((size_t)k2 * n * 8);
  L.tau = cv.take((size_t)n * 8);
  if (refine > 0) {
    L.r = cv.take((size_t)d * nrhs * 8);
    L.yr = cv.take((size_t)k * nrhs * 8);
    L.zr = cv.take((size_t)k2 * nrhs * 8);
    L.gv = cv.take(gemv64_partial_bytes(k2, nrhs, k));
    L.dx = cv.take((size_t)n * nrhs * 8);
  }
  L.total = cv.off;
  return L;
}

// rand_cholQR least squares: the multisketch of A alone, its QR (R0 kept),
// R0^{-1}, the fused pass's per-workgroup partials and their sum; for wide
// problems (n > 64 or n + nrhs > 80) R0^{-1} of order n, Q0 = A R0^{-1}
// (d x n FP64), the wide Gram pass's per-chunk partials, the Gram matrix and
// the factorisation's breakdown flag.
struct RcqLayout {
  CsLayout cs;
  size_t y = 0, partials = 0, z64 = 0, qr = 0, fact = 0, tau = 0;
  size_t r0 = 0, rinv = 0, part = 0, w = 0, q0 = 0, bad = 0, total = 0;
  bool wide = false;
};

bool rcq_is_wide(int64_t n, int64_t nrhs) {
  return n > kRcqMaxN || nrhs > kRcqMaxRhs || n + nrhs > kRcqMaxCols;
}
bool rcq_fits_wide(int64_t n, int64_t nrhs) {
  return n <= kWideMaxN && nrhs <= kWideMaxRhs && n + nrhs <= kWideMaxCols;
}

RcqLayout rcq_layout(int64_t d, int64_t n, int64_t nrhs, int64_t k, int64_t k2,
                     ms_dtype a_dtype, ms_dtype g_dtype, int mode) {
  RcqLayout L;
  Carve cv;
  carve_cs(cv, L.cs, d, k, mode, n, dtype_size(a_dtype));
  L.y = cv.take((size_t)k * n * dtype_size(a_dtype));
  L.partials = cv.take(plan_gemm(k2, n, k, g_dtype).partial_bytes);
  L.z64 = cv.take((size_t)k2 * n * 8);
  L.qr = cv.take(qr_workspace_bytes(k2, n, 0));
  L.fact = cv.take((size_t)k2 * n * 8);
  L.tau = cv.take((size_t)n * 8);
  L.wide = rcq_is_wide(n, nrhs) && rcq_fits_wide(n, nrhs);
  if (L.wide) {
    const int nc = (int)(n + nrhs);
    L.rinv = cv.take((size_t)n * n * 8);
    L.q0 = cv.take((size_t)d * n * 8);
    L.part = cv.take(gram_wide_partial_bytes(d, nc));
    L.w = cv.take(gram_wide_w_bytes(nc));
    L.bad = cv.take(4);
  } else {
    L.r0 = cv.take((size_t)kRcqMaxN * kRcqMaxN * 8);
    L.rinv = cv.take((size_t)kRcqMaxN * kRcqMaxN * 8);
    L.part = cv.take(rcq_partial_bytes(rcq_grid()));
    L.w = cv.take((size_t)kRcqMaxN * kRcqMaxCols * 8);
  }
  L.total = cv.off;
  return L;
}

// Count + SRHT multisketch least squares: the CountSketch of [A | B], its
// SRHT (per-block partials when k1 > 8192), the FP64 sketch and the QR.
struct CsrLayout {
  CsLayout cs;
  size_t y = 0, spart = 0, z64 = 0, qr = 0, fact = 0, tau = 0, total = 0;
};

CsrLayout csr_layout(int64_t d, int64_t n, int64_t nrhs, int64_t k1, int64_t k2,
                     ms_dtype a_dtype, int mode) {
  CsrLayout L;
  Carve cv;
  const int64_t nc = n + nrhs;
  carve_cs(cv, L.cs, d, k1, mode, nc, dtype_size(a_dtype));
  L.y = cv.take((size_t)k1 * nc * dtype_size(a_dtype));
  L.spart = cv.take(srht_workspace_bytes(k1, nc, k2));
  L.z64 = cv.take((size_t)k2 * nc * 8);
  L.qr = cv.take(qr_workspace_bytes(k2, n, nrhs));
  L.fact = cv.take((size_t)k2 * n * 8);
  L.tau = cv.take((size_t)n * 8);
  L.total = cv.off;
  return L;
}

// Normal equations: the fused pass's per-workgroup partials and their sum
// (n <= 64); for wider problems the wide Gram pass's per-chunk partials, the
// Gram matrix and the factorisation's breakdown flag.
struct NeLayout {
  size_t part = 0, w = 0, bad = 0, total = 0;
};

bool ne_is_wide(int64_t n, int64_t nrhs) { return rcq_is_wide(n, nrhs); }
bool ne_fits_wide(int64_t n, int64_t nrhs) { return rcq_fits_wide(n, nrhs); }

NeLayout ne_layout(int64_t d, int64_t n, int64_t nrhs) {
  NeLayout L;
  Carve cv;
  if (ne_is_wide(n, nrhs) && ne_fits_wide(n, nrhs)) {
    L.part = cv.take(gram_wide_partial_bytes(d, (int)(n + nrhs)));
    L.w = cv.take(gram_wide_w_bytes((int)(n + nrhs)));
    L.bad = cv.take(4);
  } else {
    L.part = cv.take(rcq_partial_bytes(rcq_grid()));
    L.w = cv.take((size_t)kRcqMaxN * kRcqMaxCols * 8);
  }
  L.total = cv.off;
  return L;
}

template <typename P>
P *at(void *ws, size_t off) {
  return reinterpret_cast<P *>(static_cast<unsigned char *>(ws) + off);
}

ms_status from_hip(hipError_t e) { return e == hipSuccess ? MS_OK : MS_ERR_DEVICE; }

// Sorted mode validates s with a separate pass (the plan only reads h).
__global__ void k_check_signs(int64_t d, const int8_t *__restrict__ s, int *status) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !(s[i] == 1 || s[i] == -1);
  if (bad) record_status(status, MS_ERR_RANGE);
}

hipError_t launch_check_signs(int64_t d, const int8_t *s, int *status, hipStream_t st) {
  if (d <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((d + 255) / 256, 4096);
  hipLaunchKernelGGL(k_check_signs, dim3((unsigned)blocks), dim3(256), 0, st, d, s, status);
  return hipGetLastError();
}

// CountSketch of the column set `c` into Y (k x c.ncols, ldy).  This is the
// first work of a call: its first launch also clears the status word.
//   lds    : prologue (status, Y = 0), pack h/s into validated 32-bit codes,
//            the LDS kernel (one code read per row per column tile);
//   atomic : prologue, pack, one atomic per element;
//   sorted : prologue (status, bucket counts = 0), sign check, plan, fold.
template <typename T>
hipError_t run_countsketch(int64_t d, int64_t k, const Cols<T> &c, const int32_t *h,
                           const int8_t *s, T *Y, int64_t ldy, int mode, void *ws,
                           const CsLayout &L, int *status, hipStream_t st,
                           const CsTuning &tune) {
  if (c.ncols <= 0 || d == 0)
    return launch_prologue<T>(status, Y, k, c.ncols > 0 ? c.ncols : 0, ldy, st);
  hipError_t e;
  if (mode == MS_CS_SORTED && L.bkeys_bytes) {
    e = launch_zero_status(status, st);
    if (e == hipSuccess) e = launch_bf_keys(d, k, h, s, at<uint32_t>(ws, L.bkeys), status, st);
    if (e == hipSuccess) e = launch_bf_fold<T>(d, k, c, at<uint32_t>(ws, L.bkeys), Y, ldy, st);
    return e;
  }
  if (mode == MS_CS_SORTED) {
    e = launch_prologue<int32_t>(status, at<int32_t>(ws, L.cnt), k, 1, k, st);
    if (e == hipSuccess) e = launch_check_signs(d, s, status, st);
    if (e == hipSuccess)
      e = L.tab_bytes
              ? launch_plan_blocked(d, k, h, s, at<int32_t>(ws, L.cnt), at<int32_t>(ws, L.off),
                                    at<int32_t>(ws, L.cursor), at<void>(ws, L.tab),
                                    at<uint32_t>(ws, L.sperm), status, st)
              : launch_plan(d, k, h, s, at<int32_t>(ws, L.cnt), at<int32_t>(ws, L.off),
                            at<int32_t>(ws, L.cursor), at<uint32_t>(ws, L.sperm), status, st);
    if (e != hipSuccess) return e;
    return launch_cs_sorted_cols<T>(k, c, at<int32_t>(ws, L.off), at<uint32_t>(ws, L.sperm), Y,
                                    ldy, st);
  }
  e = launch_prologue<T>(status, Y, k, c.ncols, ldy, st);
  if (e == hipSuccess && mode == MS_CS_LDS && use_tiled(L, d, k, tune)) {
    e = launch_tile_plan(d, k, nullptr, h, s, at<void>(ws, L.tplan), status, st);
    if (e == hipSuccess) e = launch_cs_tiled<T>(d, k, c, at<void>(ws, L.tplan), Y, ldy, st);
    return e;
  }
  if (e == hipSuccess) e = launch_pack_codes(d, k, h, s, at<uint32_t>(ws, L.code), status, st);
  if (e != hipSuccess) return e;
  if (mode == MS_CS_ATOMIC)
    return launch_cs_atomic<T>(d, k, c, at<uint32_t>(ws, L.code), Y, ldy, false, status, st);
  return launch_cs_lds<T>(d, k, c, at<uint32_t>(ws, L.code), nullptr, nullptr, Y, ldy, false,
                          status, st, &tune, L.part_bytes ? at<void>(ws, L.part) : nullptr,
                          L.part_bytes);
}

bool valid_mode(const ms_opts *o) {
  const int m = o ? o->cs_mode : MS_CS_AUTO;
  if (!(m >= MS_CS_AUTO && m <= MS_CS_SORTED)) return false;
  if (o && (o->cs_tile_cols < 0 || o->cs_tile_cols > 64 || o->cs_schedule < 0 || o->cs_schedule > 1))
    return false;
  if (o && !(o->gauss_y_terms == 0 || o->gauss_y_terms == 1 || o->gauss_y_terms == 3))
    return false;
  return true;
}

// BF16 terms of Y in the Gaussian stage (default: the exact three-term split)
int yterms_of(const ms_opts *o) { return (o && o->gauss_y_terms == 1) ? 1 : 3; }

CsTuning tuning_of(const ms_opts *o) {
  CsTuning t{0, 0};
  if (o) {
    t.cols_per_wg = o->cs_tile_cols;
    t.grid_variant = o->cs_schedule;
  }
  return t;
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" {

const char *ms_status_string(ms_status st) {
  switch (st) {
    case MS_OK: return "MS_OK";
    case MS_ERR_ARG: return "MS_ERR_ARG: invalid argument";
    case MS_ERR_RANGE: return "MS_ERR_RANGE: bucket index outside [0,k) or sign not +-1";
    case MS_ERR_NOMEM: return "MS_ERR_NOMEM: workspace too small";
    case MS_ERR_SINGULAR: return "MS_ERR_SINGULAR: zero or non-finite diagonal of R";
    case MS_ERR_DEVICE: return "MS_ERR_DEVICE: HIP runtime or launch failure";
    case MS_ERR_UNSUPPORTED: return "MS_ERR_UNSUPPORTED: unsupported combination or size";
  }
  return "unknown status";
}

size_t ms_workspace_size(int op, int64_t d, int64_t n, int64_t nrhs, int64_t k, int64_t k2,
                         ms_dtype a_dtype, ms_dtype g_dtype, const ms_opts *opts) {
  if (d < 0 || n < 0 || nrhs < 0 || k < 0 || k2 < 0 || !valid_mode(opts)) return 0;
  const int mode = resolve_mode(opts);
  Carve cv;
  CsLayout L;
  switch (op) {
    case MS_OP_BUCKET_PLAN:
      cv.take((size_t)k * 4);
      cv.take((size_t)d * 4);
      if (plan_blocked_bytes(d, k)) cv.take(plan_blocked_bytes(d, k));
      return cv.off;
    case MS_OP_COUNTSKETCH:
      carve_cs(cv, L, d, k, mode, n, dtype_size(a_dtype));
      return cv.off;
    case MS_OP_GAUSSIAN:
      cv.take(plan_gemm(k2, n, k, g_dtype).partial_bytes);
      return cv.off;
    case MS_OP_MULTISKETCH:
      carve_cs(cv, L, d, k, mode, n, dtype_size(a_dtype));
      cv.take((size_t)k * n * dtype_size(a_dtype));
      cv.take(plan_gemm(k2, n, k, g_dtype).partial_bytes);
      return cv.off;
    case MS_OP_QR_SOLVE:
      cv.take(qr_workspace_bytes(k2, n, nrhs));
      return cv.off;
    case MS_OP_LSTSQ: {
      const int refine = opts ? opts->refine_steps : 0;
      return lstsq_layout(d, n, nrhs, k, k2, a_dtype, g_dtype, mode, refine).total;
    }
    case MS_OP_RAND_CHOLQR:
      return rcq_layout(d, n, nrhs, k, k2, a_dtype, g_dtype, mode).total;
    case MS_OP_NORMAL_EQUATIONS:
      return ne_layout(d, n, nrhs).total;
    case MS_OP_SRHT:
      cv.take(srht_workspace_bytes(d, n, k));
      return cv.off;
    case MS_OP_COUNT_SRHT_LSTSQ:
      return csr_layout(d, n, nrhs, k, k2, a_dtype, mode).total;
    case MS_OP_COUNTSKETCH_HASHED: {
      const size_t pb = cs_part_bytes(d, k, n, dtype_size(a_dtype));
      if (pb) cv.take(pb);
      return cv.off;
    }
    default:
      return 0;
  }
}

ms_status ms_check_status(const void *ws, void *stream) {
  if (!ws) return MS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  int v = 0;
  if (hipMemcpyAsync(&v, ws, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    return MS_ERR_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return MS_ERR_DEVICE;
  return (ms_status)v;
}

ms_status ms_bucket_plan(int64_t d, int64_t k, const int32_t *h, int32_t *cnt, int32_t *off,
                         int32_t *perm, void *ws, size_t ws_bytes, void *stream) {
  if (d < 0 || d > kMax31 || k < 1 || k > kMax31) return MS_ERR_ARG;
  if ((d > 0 && (!h || !perm)) || !cnt || !off || !ws) return MS_ERR_ARG;
  const size_t need = ms_workspace_size(MS_OP_BUCKET_PLAN, d, 0, 0, k, 0, MS_F64, MS_F64, nullptr);
  if (ws_bytes < need) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  Carve cv;
  const size_t o_cursor = cv.take((size_t)k * 4);
  const size_t o_sperm = cv.take((size_t)d * 4);
  const size_t tab_bytes = d > 0 ? plan_blocked_bytes(d, k) : 0;
  const size_t o_tab = tab_bytes ? cv.take(tab_bytes) : 0;
  int *status = static_cast<int *>(ws);
  hipError_t e = launch_prologue<int32_t>(status, cnt, k, 1, k, st);
  if (tab_bytes) {
    // with no signs given the blocked plan's entries are the row indices
    // themselves: it writes the permutation in place
    if (e == hipSuccess)
      e = launch_plan_blocked(d, k, h, nullptr, cnt, off, at<int32_t>(ws, o_cursor),
                              at<void>(ws, o_tab), reinterpret_cast<uint32_t *>(perm), status, st);
    return from_hip(e);
  }
  if (e == hipSuccess)
    e = launch_plan(d, k, h, nullptr, cnt, off, at<int32_t>(ws, o_cursor),
                    at<uint32_t>(ws, o_sperm), status, st);
  if (e == hipSuccess) e = launch_strip_sign(d, at<uint32_t>(ws, o_sperm), perm, st);
  return from_hip(e);
}

ms_status ms_pack_sketch(int64_t d, int64_t k, const int32_t *h, const int8_t *s, uint32_t *code,
                         void *ws, size_t ws_bytes, void *stream) {
  if (d < 0 || k < 1 || k > kMax31) return MS_ERR_ARG;
  if (!ws || ws_bytes < kAlign || (d > 0 && (!h || !s || !code))) return MS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  hipError_t e = launch_zero_status(status, st);
  if (e == hipSuccess) e = launch_pack_codes(d, k, h, s, code, status, st);
  return from_hip(e);
}

ms_status countsketch_accumulate(int64_t d, int64_t n, int64_t k, ms_dtype a_dtype, const void *A,
                                 int64_t lda, const uint32_t *code, void *Y, int64_t ldy,
                                 const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  if (d < 0 || n < 0 || k < 1 || k > kMax31 || n > (int64_t)1 << 30) return MS_ERR_ARG;
  if (a_dtype != MS_F64 && a_dtype != MS_F32) return MS_ERR_ARG;
  if (!valid_mode(opts)) return MS_ERR_ARG;
  const int mode = resolve_mode(opts);
  if (mode == MS_CS_SORTED) return MS_ERR_UNSUPPORTED;
  if (lda < (d > 1 ? d : 1) || ldy < k) return MS_ERR_ARG;
  if (!ws || ws_bytes < kAlign || (n > 0 && !Y) || (d > 0 && n > 0 && (!A || !code)))
    return MS_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  hipError_t e = launch_zero_status(status, st);
  if (e != hipSuccess || n == 0 || d == 0) return from_hip(e);
  const CsTuning tune = tuning_of(opts);
  // a workspace beyond the status block holds the tiled CountSketch's plan
  // (k > 16384), built here from the codes
  const size_t tneed = cs_tile_plan_bytes(d, k);
  if (mode == MS_CS_LDS && tneed && ws_bytes >= kAlign + tneed && !tune.grid_variant &&
      !tune.cols_per_wg && cs_tiled_supported(d, k)) {
    void *plan = at<void>(ws, kAlign);
    e = launch_tile_plan(d, k, code, nullptr, nullptr, plan, status, st);
    if (e != hipSuccess) return from_hip(e);
    if (a_dtype == MS_F64) {
      Cols<double> c{static_cast<const double *>(A), lda, nullptr, 0, (int)n, (int)n};
      e = launch_cs_tiled<double>(d, k, c, plan, static_cast<double *>(Y), ldy, st);
    } else {
      Cols<float> c{static_cast<const float *>(A), lda, nullptr, 0, (int)n, (int)n};
      e = launch_cs_tiled<float>(d, k, c, plan, static_cast<float *>(Y), ldy, st);
    }
    return from_hip(e);
  }
  // else a workspace beyond the status block holds the per-die partial buffer
  const size_t pneed = cs_part_bytes(d, k, n, dtype_size(a_dtype));
  void *part = (pneed && ws_bytes >= kAlign + pneed) ? at<void>(ws, kAlign) : nullptr;
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = mode == MS_CS_ATOMIC
            ? launch_cs_atomic<double>(d, k, c, code, static_cast<double *>(Y), ldy, false, status, st)
            : launch_cs_lds<double>(d, k, c, code, nullptr, nullptr, static_cast<double *>(Y), ldy,
                                    false, status, st, &tune, part, part ? pneed : 0);
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = mode == MS_CS_ATOMIC
            ? launch_cs_atomic<float>(d, k, c, code, static_cast<float *>(Y), ldy, false, status, st)
            : launch_cs_lds<float>(d, k, c, code, nullptr, nullptr, static_cast<float *>(Y), ldy,
                                   false, status, st, &tune, part, part ? pneed : 0);
  }
  return from_hip(e);
}

ms_status countsketch_apply(int64_t d, int64_t n, int64_t k, ms_dtype a_dtype, const void *A,
                            int64_t lda, const int32_t *h, const int8_t *s, void *Y, int64_t ldy,
                            const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  if (d < 0 || n < 0 || k < 1 || k > kMax31 || n > (int64_t)1 << 30) return MS_ERR_ARG;
  if (a_dtype != MS_F64 && a_dtype != MS_F32) return MS_ERR_ARG;
  if (!valid_mode(opts)) return MS_ERR_ARG;
  const int mode = resolve_mode(opts);
  if (mode == MS_CS_SORTED && d > kMax31) return MS_ERR_UNSUPPORTED;
  if (lda < (d > 1 ? d : 1) || ldy < k) return MS_ERR_ARG;
  if (!ws || (n > 0 && !Y) || (d > 0 && n > 0 && (!A || !h || !s))) return MS_ERR_ARG;
  if (ws_bytes < ms_workspace_size(MS_OP_COUNTSKETCH, d, n, 0, k, 0, a_dtype, a_dtype, opts))
    return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  if (n == 0) return from_hip(launch_zero_status(status, st));
  hipError_t e;
  Carve cv;
  CsLayout L;
  carve_cs(cv, L, d, k, mode, n, dtype_size(a_dtype));
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = run_countsketch<double>(d, k, c, h, s, static_cast<double *>(Y), ldy, mode, ws, L, status,
                                st, tuning_of(opts));
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = run_countsketch<float>(d, k, c, h, s, static_cast<float *>(Y), ldy, mode, ws, L, status,
                               st, tuning_of(opts));
  }
  return from_hip(e);
}

ms_status ms_gaussian_apply(int64_t k, int64_t ncols, int64_t k2, ms_dtype g_dtype, const void *G,
                            int64_t ldg, ms_dtype y_dtype, const void *Y, int64_t ldy, void *Z,
                            int64_t ldz, void *ws, size_t ws_bytes, void *stream) {
  if (k < 1 || ncols < 0 || k2 < 1 || k2 > (1 << 24) || ncols > (1 << 24)) return MS_ERR_ARG;
  const bool ok = (g_dtype == MS_F64 && y_dtype == MS_F64) ||
                  (g_dtype == MS_F32 && y_dtype == MS_F32) ||
                  ((g_dtype == MS_BF16 || g_dtype == MS_F16) && y_dtype == MS_F32);
  if (!ok) return MS_ERR_ARG;
  if (ldg < k2 || ldy < k || ldz < k2) return MS_ERR_ARG;
  if (!ws || (ncols > 0 && (!G || !Y || !Z))) return MS_ERR_ARG;
  if (ws_bytes < ms_workspace_size(MS_OP_GAUSSIAN, 0, ncols, 0, k, k2, y_dtype, g_dtype, nullptr))
    return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_zero_status(static_cast<int *>(ws), st);
  if (e != hipSuccess || ncols == 0) return from_hip(e);
  Carve cv;
  const GemmPlan p = plan_gemm(k2, ncols, k, g_dtype);
  const size_t o_part = cv.take(p.partial_bytes);
  e = launch_gemm(p, g_dtype, G, ldg, Y, ldy, Z, ldz, nullptr, at<void>(ws, o_part), nullptr, st);
  return from_hip(e);
}

ms_status multisketch_apply(int64_t d, int64_t n, int64_t k, int64_t k2, ms_dtype a_dtype,
                            const void *A, int64_t lda, const int32_t *h, const int8_t *s,
                            ms_dtype g_dtype, const void *G, int64_t ldg, void *Z, int64_t ldz,
                            const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  if (d < 0 || n < 0 || k < 1 || k > kMax31 || k2 < 1 || k2 > (1 << 24) || n > (1 << 24))
    return MS_ERR_ARG;
  const bool ok = (a_dtype == MS_F64 && g_dtype == MS_F64) ||
                  (a_dtype == MS_F32 &&
                   (g_dtype == MS_F32 || g_dtype == MS_BF16 || g_dtype == MS_F16));
  if (!ok || !valid_mode(opts)) return MS_ERR_ARG;
  const int mode = resolve_mode(opts);
  if (mode == MS_CS_SORTED && d > kMax31) return MS_ERR_UNSUPPORTED;
  if (lda < (d > 1 ? d : 1) || ldg < k2 || ldz < k2) return MS_ERR_ARG;
  if (!ws || (n > 0 && (!Z || !G)) || (d > 0 && n > 0 && (!A || !h || !s))) return MS_ERR_ARG;
  if (ws_bytes < ms_workspace_size(MS_OP_MULTISKETCH, d, n, 0, k, k2, a_dtype, g_dtype, opts))
    return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  if (n == 0) return from_hip(launch_zero_status(status, st));
  hipError_t e;
  Carve cv;
  CsLayout L;
  carve_cs(cv, L, d, k, mode, n, dtype_size(a_dtype));
  const size_t o_y = cv.take((size_t)k * n * dtype_size(a_dtype));
  const GemmPlan p = plan_gemm(k2, n, k, g_dtype);
  const size_t o_part = cv.take(p.partial_bytes);
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = run_countsketch<double>(d, k, c, h, s, at<double>(ws, o_y), k, mode, ws, L, status, st, tuning_of(opts));
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = run_countsketch<float>(d, k, c, h, s, at<float>(ws, o_y), k, mode, ws, L, status, st, tuning_of(opts));
  }
  if (e == hipSuccess)
    e = launch_gemm(p, g_dtype, G, ldg, at<void>(ws, o_y), k, Z, ldz, nullptr,
                    at<void>(ws, o_part), nullptr, st, yterms_of(opts));
  return from_hip(e);
}

ms_status ms_qr_solve(int64_t m, int64_t n, int64_t nrhs, const double *W, int64_t ldw,
                      const double *Bm, int64_t ldb, double *X, int64_t ldx, double *R,
                      int64_t ldr, void *ws, size_t ws_bytes, void *stream) {
  if (n < 1 || m < n || nrhs < 0 || m > (1 << 24) || n > (1 << 16) || nrhs > (1 << 16))
    return MS_ERR_ARG;
  if (ldw < m || (nrhs > 0 && ldb < m) || ldx < n || (R && ldr < n)) return MS_ERR_ARG;
  if (!W || !ws || (nrhs > 0 && (!Bm || !X))) return MS_ERR_ARG;
  if (ws_bytes < ms_workspace_size(MS_OP_QR_SOLVE, 0, n, nrhs, 0, m, MS_F64, MS_F64, nullptr))
    return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  hipError_t e = launch_zero_status(status, st);
  Carve cv;
  const size_t o_qr = cv.take(qr_workspace_bytes(m, n, nrhs));
  if (e == hipSuccess)
    e = launch_qr_solve(m, n, nrhs, W, ldw, Bm, ldb, X, ldx, R, ldr, nullptr, nullptr,
                        at<void>(ws, o_qr), status, st);
  return from_hip(e);
}

ms_status sketch_lstsq(int64_t d, int64_t n, int64_t nrhs, int64_t k, int64_t k2,
                       ms_dtype a_dtype, const void *A, int64_t lda, const void *B, int64_t ldb,
                       const int32_t *h, const int8_t *s, ms_dtype g_dtype, const void *G,
                       int64_t ldg, double *X, int64_t ldx, const ms_opts *opts, void *ws,
                       size_t ws_bytes, void *stream) {
  if (d < 1 || n < 1 || nrhs < 1 || k < 1 || k > kMax31 || k2 < n || k2 > (1 << 24) ||
      n > (1 << 16) || nrhs > (1 << 16))
    return MS_ERR_ARG;
  const bool ok = (a_dtype == MS_F64 && g_dtype == MS_F64) ||
                  (a_dtype == MS_F32 &&
                   (g_dtype == MS_F32 || g_dtype == MS_BF16 || g_dtype == MS_F16));
  if (!ok || !valid_mode(opts)) return MS_ERR_ARG;
  const int mode = resolve_mode(opts);
  const int refine = opts ? opts->refine_steps : 0;
  if (refine < 0 || refine > 64) return MS_ERR_ARG;
  if (refine > 0 && nrhs > 8) return MS_ERR_UNSUPPORTED;
  if (mode == MS_CS_SORTED && d > kMax31) return MS_ERR_UNSUPPORTED;
  if (lda < d || ldb < d || ldg < k2 || ldx < n) return MS_ERR_ARG;
  if (!A || !B || !h || !s || !G || !X || !ws) return MS_ERR_ARG;
  const LstsqLayout L = lstsq_layout(d, n, nrhs, k, k2, a_dtype, g_dtype, mode, refine);
  if (ws_bytes < L.total) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  const int64_t nc = n + nrhs;
  hipError_t e;
  // 1. Y = C [A | B]
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, static_cast<const double *>(B), ldb,
                   (int)n, (int)nc};
    e = run_countsketch<double>(d, k, c, h, s, at<double>(ws, L.y), k, mode, ws, L.cs, status, st, tuning_of(opts));
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, static_cast<const float *>(B), ldb, (int)n,
                  (int)nc};
    e = run_countsketch<float>(d, k, c, h, s, at<float>(ws, L.y), k, mode, ws, L.cs, status, st, tuning_of(opts));
  }
  // 2. Z = G Y (split-K partials reduced in split order into an FP64 Z);
  // 3. Householder QR of Z_A, Q^T Z_B, back substitution
  const GemmPlan p = plan_gemm(k2, nc, k, g_dtype);
  double *z64 = at<double>(ws, L.z64);
  if (e == hipSuccess)
    e = launch_gemm(p, g_dtype, G, ldg, at<void>(ws, L.y), k, nullptr, k2, z64,
                    at<void>(ws, L.partials), nullptr, st, yterms_of(opts));
  if (e == hipSuccess)
    e = launch_qr_solve(k2, n, nrhs, z64, k2, z64 + n * k2, k2, X, ldx, nullptr, 0,
                        at<double>(ws, L.tau), at<double>(ws, L.fact), at<void>(ws, L.qr), status,
                        st);
  // 4. refinement: r = B - A X (FP64); X += R^{-1} Q^T G (C r)
  for (int it = 0; it < refine && e == hipSuccess; ++it) {
    double *r = at<double>(ws, L.r);
    if (a_dtype == MS_F32)
      e = launch_residual_f32(d, n, nrhs, static_cast<const float *>(A), lda,
                              static_cast<const float *>(B), ldb, X, ldx, r, d, st);
    else
      e = launch_residual_f64(d, n, nrhs, static_cast<const double *>(A), lda,
                              static_cast<const double *>(B), ldb, X, ldx, r, d, st);
    if (e != hipSuccess) break;
    Cols<double> cr{r, d, nullptr, 0, (int)nrhs, (int)nrhs};
    if (mode == MS_CS_SORTED && L.cs.bkeys_bytes)
      e = launch_bf_fold<double>(d, k, cr, at<uint32_t>(ws, L.cs.bkeys), at<double>(ws, L.yr), k,
                                 st);
    else if (mode == MS_CS_SORTED)
      e = launch_cs_sorted_cols<double>(k, cr, at<int32_t>(ws, L.cs.off), at<uint32_t>(ws, L.cs.sperm),
                                   at<double>(ws, L.yr), k, st);
    else if (mode == MS_CS_ATOMIC)
      e = launch_cs_atomic<double>(d, k, cr, at<uint32_t>(ws, L.cs.code), at<double>(ws, L.yr), k,
                                   true, status, st);
    else if (use_tiled(L.cs, d, k, tuning_of(opts))) {
      e = launch_fill_zero<double>(at<double>(ws, L.yr), k, nrhs, k, st);
      if (e == hipSuccess)
        e = launch_cs_tiled<double>(d, k, cr, at<void>(ws, L.cs.tplan), at<double>(ws, L.yr), k,
                                    st);
    } else
      e = launch_cs_lds<double>(d, k, cr, at<uint32_t>(ws, L.cs.code), nullptr, nullptr,
                                at<double>(ws, L.yr), k, true, status, st);
    if (e != hipSuccess) break;
    e = launch_gemv64(k2, nrhs, k, g_dtype, G, ldg, at<double>(ws, L.yr), k, at<double>(ws, L.zr),
                      at<double>(ws, L.gv), st);
    if (e != hipSuccess) break;
    e = launch_qr_apply_solve(k2, n, nrhs, at<double>(ws, L.fact), at<double>(ws, L.tau),
                              at<double>(ws, L.zr), at<double>(ws, L.dx), n, status, st);
    if (e != hipSuccess) break;
    e = launch_axpy_update(n, nrhs, at<double>(ws, L.dx), X, ldx, st);
  }
  return from_hip(e);
}

ms_status rand_cholqr_lstsq(int64_t d, int64_t n, int64_t nrhs, int64_t k, int64_t k2,
                            ms_dtype a_dtype, const void *A, int64_t lda, const void *B,
                            int64_t ldb, const int32_t *h, const int8_t *s, ms_dtype g_dtype,
                            const void *G, int64_t ldg, double *X, int64_t ldx, double *R,
                            int64_t ldr, const ms_opts *opts, void *ws, size_t ws_bytes,
                            void *stream) {
  if (d < 1 || n < 1 || nrhs < 1 || k < 1 || k > kMax31 || k2 < n || k2 > (1 << 24))
    return MS_ERR_ARG;
  const bool ok = (a_dtype == MS_F64 && g_dtype == MS_F64) ||
                  (a_dtype == MS_F32 &&
                   (g_dtype == MS_F32 || g_dtype == MS_BF16 || g_dtype == MS_F16));
  if (!ok || !valid_mode(opts)) return MS_ERR_ARG;
  if (opts && opts->refine_steps != 0) return MS_ERR_ARG;
  if (rcq_is_wide(n, nrhs) && !rcq_fits_wide(n, nrhs)) return MS_ERR_UNSUPPORTED;
  const int mode = resolve_mode(opts);
  if (mode == MS_CS_SORTED && d > kMax31) return MS_ERR_UNSUPPORTED;
  if (lda < d || ldb < d || ldg < k2 || ldx < n || (R && ldr < n)) return MS_ERR_ARG;
  if (!A || !B || !h || !s || !G || !X || !ws) return MS_ERR_ARG;
  const RcqLayout L = rcq_layout(d, n, nrhs, k, k2, a_dtype, g_dtype, mode);
  if (ws_bytes < L.total) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  hipError_t e;
  // 1. Y = S A (CountSketch of A, then the Gaussian stage into an FP64 Z)
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = run_countsketch<double>(d, k, c, h, s, at<double>(ws, L.y), k, mode, ws, L.cs, status,
                                st, tuning_of(opts));
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, nullptr, 0, (int)n, (int)n};
    e = run_countsketch<float>(d, k, c, h, s, at<float>(ws, L.y), k, mode, ws, L.cs, status, st,
                               tuning_of(opts));
  }
  const GemmPlan p = plan_gemm(k2, n, k, g_dtype);
  double *z64 = at<double>(ws, L.z64);
  if (e == hipSuccess)
    e = launch_gemm(p, g_dtype, G, ldg, at<void>(ws, L.y), k, nullptr, k2, z64,
                    at<void>(ws, L.partials), nullptr, st, yterms_of(opts));
  double *fact = at<double>(ws, L.fact), *rinv = at<double>(ws, L.rinv);
  if (L.wide) {
    // 2. R0: the upper part of the QR factors of S A (ld k2)
    if (e == hipSuccess)
      e = launch_qr_solve(k2, n, 0, z64, k2, nullptr, k2, X, ldx, nullptr, 0,
                          at<double>(ws, L.tau), fact, at<void>(ws, L.qr), status, st);
    // 3. R0^{-1} and Q0 = A R0^{-1}
    double *q0 = at<double>(ws, L.q0);
    if (e == hipSuccess)
      e = launch_rcq_wide_q0(d, (int)n, a_dtype, A, lda, fact, k2, rinv, q0, status, st);
    // 4. W = [Q0 | B]^T [Q0 | B]
    const int nc = (int)(n + nrhs);
    double *part = at<double>(ws, L.part), *W = at<double>(ws, L.w);
    if (e == hipSuccess)
      e = a_dtype == MS_F64
              ? launch_gram_wide<double, double>(d, (int)n, nc, q0, d,
                                                 static_cast<const double *>(B), ldb, part, W, st)
              : launch_gram_wide<double, float>(d, (int)n, nc, q0, d,
                                                static_cast<const float *>(B), ldb, part, W, st);
    // 5-8. R1 = chol(Q0^T Q0), y = R1^{-T} Q0^T B, x = R0^{-1} R1^{-1} y, R = R1 R0
    if (e == hipSuccess)
      e = launch_chol_solve_wide((int)n, (int)nrhs, nc, W, fact, k2, X, ldx, R, ldr,
                                 at<int>(ws, L.bad), status, st);
    return from_hip(e);
  }
  // 2. R0 of the Householder QR of S A (no right-hand side)
  double *r0 = at<double>(ws, L.r0);
  if (e == hipSuccess)
    e = launch_qr_solve(k2, n, 0, z64, k2, nullptr, k2, X, ldx, r0, kRcqMaxN,
                        at<double>(ws, L.tau), fact, at<void>(ws, L.qr), status, st);
  // 3-4. R0^{-1}; one pass: Q0 = A R0^{-1}, per-workgroup Q0^T [Q0 | B]
  double *part = at<double>(ws, L.part);
  const int grid = rcq_grid();
  if (e == hipSuccess) e = launch_rcq_trinv((int)n, r0, kRcqMaxN, rinv, status, st);
  if (e == hipSuccess)
    e = a_dtype == MS_F64
            ? launch_rcq_gram<double>(d, (int)n, (int)nrhs, static_cast<const double *>(A), lda,
                                      static_cast<const double *>(B), ldb, rinv, part, grid, st)
            : launch_rcq_gram<float>(d, (int)n, (int)nrhs, static_cast<const float *>(A), lda,
                                     static_cast<const float *>(B), ldb, rinv, part, grid, st);
  // 5-8. the partials' sum, R1 = chol(Q0^T Q0), R = R1 R0, y = R1^{-T} Q0^T B,
  // x = R^{-1} y
  if (e == hipSuccess)
    e = launch_rcq_finish((int)n, (int)nrhs, grid, part, at<double>(ws, L.w), r0, kRcqMaxN, rinv,
                          X, ldx, R, ldr, status, st);
  return from_hip(e);
}

ms_status countsketch_hashed(int64_t d, int64_t n, int64_t k, uint64_t seed, ms_dtype a_dtype,
                             const void *A, int64_t lda, void *Y, int64_t ldy,
                             const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  if (d < 0 || n < 0 || k < 1 || k > kMax31 || n > (int64_t)1 << 30) return MS_ERR_ARG;
  if (a_dtype != MS_F64 && a_dtype != MS_F32) return MS_ERR_ARG;
  if (!valid_mode(opts)) return MS_ERR_ARG;
  const int m = opts ? opts->cs_mode : MS_CS_AUTO;
  if ((m != MS_CS_AUTO && m != MS_CS_LDS) || (opts && opts->cs_schedule != 0))
    return MS_ERR_UNSUPPORTED;
  if (lda < (d > 1 ? d : 1) || ldy < k) return MS_ERR_ARG;
  if (!ws || (n > 0 && !Y) || (d > 0 && n > 0 && !A)) return MS_ERR_ARG;
  const size_t need = ms_workspace_size(MS_OP_COUNTSKETCH_HASHED, d, n, 0, k, 0, a_dtype, a_dtype,
                                        opts);
  if (ws_bytes < need) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  if (n == 0) return from_hip(launch_zero_status(status, st));
  Carve cv;
  const size_t pbytes = cs_part_bytes(d, k, n, dtype_size(a_dtype));
  void *part = pbytes ? at<void>(ws, cv.take(pbytes)) : nullptr;
  const CsTuning tune = tuning_of(opts);
  hipError_t e;
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, nullptr, 0, (int)n, (int)n, 1, seed};
    e = launch_prologue<double>(status, static_cast<double *>(Y), k, n, ldy, st);
    if (e == hipSuccess)
      e = launch_cs_lds<double>(d, k, c, nullptr, nullptr, nullptr, static_cast<double *>(Y), ldy,
                                false, status, st, &tune, part, pbytes);
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, nullptr, 0, (int)n, (int)n, 1, seed};
    e = launch_prologue<float>(status, static_cast<float *>(Y), k, n, ldy, st);
    if (e == hipSuccess)
      e = launch_cs_lds<float>(d, k, c, nullptr, nullptr, nullptr, static_cast<float *>(Y), ldy,
                               false, status, st, &tune, part, pbytes);
  }
  return from_hip(e);
}

ms_status srht_apply(int64_t m, int64_t ncols, int64_t k, ms_dtype x_dtype, const void *X,
                     int64_t ldx, const int8_t *dsign, const int32_t *r, double *Y, int64_t ldy,
                     void *ws, size_t ws_bytes, void *stream) {
  if (m < 1 || m > kMax31 || ncols < 0 || ncols > 65535 || k < 1 || k > (1 << 24))
    return MS_ERR_ARG;
  if (x_dtype != MS_F64 && x_dtype != MS_F32) return MS_ERR_ARG;
  if (ldx < m || ldy < k || !ws || (ncols > 0 && (!X || !dsign || !r || !Y))) return MS_ERR_ARG;
  Carve cv;
  const size_t pbytes = srht_workspace_bytes(m, ncols, k);
  void *part = pbytes ? at<void>(ws, cv.take(pbytes)) : nullptr;
  if (ws_bytes < cv.off) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  hipError_t e = launch_zero_status(status, st);
  if (e == hipSuccess && ncols > 0)
    e = x_dtype == MS_F64
            ? launch_srht<double>(m, ncols, k, static_cast<const double *>(X), ldx, dsign, r, Y,
                                  ldy, part, status, st)
            : launch_srht<float>(m, ncols, k, static_cast<const float *>(X), ldx, dsign, r, Y, ldy,
                                 part, status, st);
  return from_hip(e);
}

ms_status count_srht_lstsq(int64_t d, int64_t n, int64_t nrhs, int64_t k1, int64_t k2,
                           ms_dtype a_dtype, const void *A, int64_t lda, const void *B,
                           int64_t ldb, const int32_t *h, const int8_t *s, const int8_t *dsign,
                           const int32_t *r, double *X, int64_t ldx, const ms_opts *opts, void *ws,
                           size_t ws_bytes, void *stream) {
  if (d < 1 || n < 1 || nrhs < 1 || k1 < 1 || k1 > kMax31 || k2 < n || k2 > (1 << 24))
    return MS_ERR_ARG;
  if (a_dtype != MS_F64 && a_dtype != MS_F32) return MS_ERR_ARG;
  if (!valid_mode(opts) || (opts && opts->refine_steps != 0)) return MS_ERR_ARG;
  if (n + nrhs > 65535) return MS_ERR_UNSUPPORTED;
  const int mode = resolve_mode(opts);
  if (mode == MS_CS_SORTED && d > kMax31) return MS_ERR_UNSUPPORTED;
  if (lda < d || ldb < d || ldx < n) return MS_ERR_ARG;
  if (!A || !B || !h || !s || !dsign || !r || !X || !ws) return MS_ERR_ARG;
  const CsrLayout L = csr_layout(d, n, nrhs, k1, k2, a_dtype, mode);
  if (ws_bytes < L.total) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  const int64_t nc = n + nrhs;
  double *z64 = at<double>(ws, L.z64);
  void *sp = L.spart ? at<void>(ws, L.spart) : nullptr;
  hipError_t e;
  // 1. Y = C [A | B] (k1 x nc, A's precision); 2. Z = SRHT(Y) (k2 x nc, FP64)
  if (a_dtype == MS_F64) {
    Cols<double> c{static_cast<const double *>(A), lda, static_cast<const double *>(B), ldb,
                   (int)n, (int)nc};
    e = run_countsketch<double>(d, k1, c, h, s, at<double>(ws, L.y), k1, mode, ws, L.cs, status,
                                st, tuning_of(opts));
    if (e == hipSuccess)
      e = launch_srht<double>(k1, nc, k2, at<double>(ws, L.y), k1, dsign, r, z64, k2, sp, status,
                              st);
  } else {
    Cols<float> c{static_cast<const float *>(A), lda, static_cast<const float *>(B), ldb, (int)n,
                  (int)nc};
    e = run_countsketch<float>(d, k1, c, h, s, at<float>(ws, L.y), k1, mode, ws, L.cs, status, st,
                               tuning_of(opts));
    if (e == hipSuccess)
      e = launch_srht<float>(k1, nc, k2, at<float>(ws, L.y), k1, dsign, r, z64, k2, sp, status,
                             st);
  }
  // 3. Householder QR of Z_A, Q^T Z_B, back substitution (FP64)
  if (e == hipSuccess)
    e = launch_qr_solve(k2, n, nrhs, z64, k2, z64 + n * k2, k2, X, ldx, nullptr, 0,
                        at<double>(ws, L.tau), at<double>(ws, L.fact), at<void>(ws, L.qr), status,
                        st);
  return from_hip(e);
}

ms_status ms_hash_sketch(int64_t d, int64_t k, uint64_t seed, int32_t *h, int8_t *s,
                         void *stream) {
  if (d < 0 || k < 1 || k > kMax31 || (d > 0 && (!h || !s))) return MS_ERR_ARG;
  return from_hip(launch_hash_sketch(d, k, seed, h, s, (hipStream_t)stream));
}

ms_status normal_equations_lstsq(int64_t d, int64_t n, int64_t nrhs, ms_dtype a_dtype,
                                 const void *A, int64_t lda, const void *B, int64_t ldb,
                                 double *X, int64_t ldx, double *R, int64_t ldr,
                                 const ms_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  (void)opts;
  if (d < 1 || n < 1 || nrhs < 1) return MS_ERR_ARG;
  if (a_dtype != MS_F64 && a_dtype != MS_F32) return MS_ERR_ARG;
  const bool wide = ne_is_wide(n, nrhs);
  if (wide && !ne_fits_wide(n, nrhs)) return MS_ERR_UNSUPPORTED;
  if (lda < d || ldb < d || ldx < n || (R && ldr < n)) return MS_ERR_ARG;
  if (!A || !B || !X || !ws) return MS_ERR_ARG;
  const NeLayout L = ne_layout(d, n, nrhs);
  if (ws_bytes < L.total) return MS_ERR_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  int *status = static_cast<int *>(ws);
  double *part = at<double>(ws, L.part);
  const int grid = rcq_grid();
  hipError_t e = launch_zero_status(status, st);
  if (wide) {
    // W = [A | B]^T [A | B] by the wide Gram pass (per-chunk partials, then
    // their ordered sum), then the blocked Cholesky and the two solves
    const int nc = (int)(n + nrhs);
    double *W = at<double>(ws, L.w);
    if (e == hipSuccess)
      e = a_dtype == MS_F64
              ? launch_gram_wide<double, double>(d, (int)n, nc, static_cast<const double *>(A), lda,
                                                 static_cast<const double *>(B), ldb, part, W, st)
              : launch_gram_wide<float, float>(d, (int)n, nc, static_cast<const float *>(A), lda,
                                               static_cast<const float *>(B), ldb, part, W, st);
    if (e == hipSuccess)
      e = launch_chol_solve_wide((int)n, (int)nrhs, nc, W, nullptr, 0, X, ldx, R, ldr,
                                 at<int>(ws, L.bad), status, st);
    return from_hip(e);
  }
  // one pass: per-workgroup [A | B]^T [A | B] (FP64), then the ordered sum,
  // R = chol(A^T A), R^T y = A^T B, X = R^{-1} y
  if (e == hipSuccess)
    e = a_dtype == MS_F64
            ? launch_rcq_gram<double>(d, (int)n, (int)nrhs, static_cast<const double *>(A), lda,
                                      static_cast<const double *>(B), ldb, nullptr, part, grid,
                                      st)
            : launch_rcq_gram<float>(d, (int)n, (int)nrhs, static_cast<const float *>(A), lda,
                                     static_cast<const float *>(B), ldb, nullptr, part, grid, st);
  if (e == hipSuccess)
    e = launch_rcq_finish((int)n, (int)nrhs, grid, part, at<double>(ws, L.w), nullptr, 0, nullptr,
                          X, ldx, R, ldr, status, st);
  return from_hip(e);
}

}  // extern "C"
