// Allocation-free least squares: the workspace and task graphs of
// tqr_lstsq live in one statically allocated device array per GPU.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tqr.h"

namespace tqr {
int lstsq_scratch(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                  int64_t ldb, double *X, int64_t ldx, const tqr_opts *o, int32_t *info, hipStream_t stream,
                  char *scratch, size_t scratch_bytes);
}

// In host code `scratch` names a host-side stand-in; its device address is
// looked up once per device (hipGetSymbolAddress) and only that address is
// ever passed to copies and kernels.
static __device__ __align__(256) unsigned char scratch[TQR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The device address of this device's scratch array (set up on the first
// call on each device, with that device current).
int scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TQR_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TQR_E_HIP;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return TQR_OK;
}
}  // namespace

extern "C" int tqr_lstsq_noalloc(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                 const double *B, int64_t ldb, double *X, int64_t ldx, const tqr_opts *o,
                                 int32_t *info, hipStream_t stream) {
  void *ptr = nullptr;
  const int rc = scratch_address(&ptr);
  if (rc) return rc;
  return tqr::lstsq_scratch(m, n, nrhs, A, lda, B, ldb, X, ldx, o, info, stream, static_cast<char *>(ptr),
                            TQR_NOALLOC_SCRATCH_BYTES);
}
