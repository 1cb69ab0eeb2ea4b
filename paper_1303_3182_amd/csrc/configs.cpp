// Tile configurations built into the library, and the dispatch from (nb, ib)
// to the per-configuration objects compiled from kernels.hip.
#include <hip/hip_runtime_api.h>

#include "tqr_types.h"

namespace tqr {

// nb, ib; the chunk width (columns of a register-resident update pass) is
// min(nb, 64) for every configuration.
#define TQR_CONFIGS(X) \
  X(32, 16)            \
  X(64, 16)            \
  X(64, 32)            \
  X(128, 32)           \
  X(256, 32)

#define X(NB, IB)                                                                                  \
  hipError_t launch_exec_##NB##_##IB(const ExecArgs &a, int mode, int grid, const int32_t *order, \
                                     int32_t *info, hipStream_t s);                              \
  int exec_occupancy_##NB##_##IB();
TQR_CONFIGS(X)
#undef X

// mode: 0 persistent, 1 sequential (one launch per task in the host-side
// topological order `order`).
hipError_t launch_exec(const ExecArgs &a, int mode, int grid, const int32_t *order, int32_t *info,
                       hipStream_t s) {
#define X(NB, IB) \
  if (a.nb == NB && a.ib == IB) return launch_exec_##NB##_##IB(a, mode, grid, order, info, s);
  TQR_CONFIGS(X)
#undef X
  return hipErrorInvalidValue;
}

int exec_occupancy(int nb, int ib) {
#define X(NB, IB) \
  if (nb == NB && ib == IB) return exec_occupancy_##NB##_##IB();
  TQR_CONFIGS(X)
#undef X
  return 0;
}

bool config_supported(int nb, int ib) {
#define X(NB, IB) \
  if (nb == NB && ib == IB) return true;
  TQR_CONFIGS(X)
#undef X
  return false;
}

int config_list(int *nb, int *ib, int cap) {
  int k = 0;
#define X(NB, IB)     \
  if (k < cap) {      \
    nb[k] = NB;       \
    ib[k] = IB;       \
  }                   \
  k++;
  TQR_CONFIGS(X)
#undef X
  return k;
}

int chunk_width(int nb, int ib) {
  (void)ib;
  return nb < 64 ? nb : 64;
}

}  // namespace tqr
