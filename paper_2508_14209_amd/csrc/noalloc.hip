// noalloc.hip -- sketch_lstsq_noalloc: the multisketch sketch-and-solve of
// sketch_lstsq for callers that cannot allocate device memory (code under
// stream capture, tight serving loops, harnesses that forbid allocation).
//
// Its scratch space is one file-scope device array per GPU, `scratch`, of
// MS_NOALLOC_SCRATCH_BYTES bytes, held by each device the library runs on
// until the process ends.  In host code the array's name is only a host-side
// stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and every use goes through
// that address.  The kernels are those of sketch_lstsq; the scratch array
// takes the place of the caller's workspace.  Calls on one GPU share its
// array: calls that overlap on that GPU (different streams without ordering)
// race on it.
#include <mutex>

#include "ms_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[MS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The device address of this device's scratch array (looked up on the first
// call on the device), or null when the lookup fails.
void *scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Copy the scratch array's status word to the caller's status output.
__global__ void k_copy_status(const int *__restrict__ src, int32_t *__restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

}  // namespace

extern "C" ms_status sketch_lstsq_noalloc(int64_t d, int64_t n, int64_t nrhs, int64_t k,
                                          int64_t k2, ms_dtype a_dtype, const void *A,
                                          int64_t lda, const void *B, int64_t ldb,
                                          const int32_t *h, const int8_t *s, ms_dtype g_dtype,
                                          const void *G, int64_t ldg, double *X, int64_t ldx,
                                          int32_t *status, const ms_opts *opts, void *stream) {
  const size_t need = ms_workspace_size(MS_OP_LSTSQ, d, n, nrhs, k, k2, a_dtype, g_dtype, opts);
  if (need == 0) return MS_ERR_ARG;
  if (need > (size_t)MS_NOALLOC_SCRATCH_BYTES) return MS_ERR_NOMEM;
  void *ws = scratch_of_current_device();
  if (!ws) return MS_ERR_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const ms_status r = sketch_lstsq(d, n, nrhs, k, k2, a_dtype, A, lda, B, ldb, h, s, g_dtype, G,
                                   ldg, X, ldx, opts, ws, (size_t)MS_NOALLOC_SCRATCH_BYTES, stream);
  if (r != MS_OK || !status) return r;
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, static_cast<const int *>(ws),
                     status);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_ERR_DEVICE;
}
