// Refinement kernels (refine.hip): FP64 residuals with compensated dot
// products, the backward-error stopping test and the correction update, for
// one problem or a batch; plus batched column-major copies.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "tqr.h"

namespace tqr {

constexpr int kRefineHistory = TQR_REFINE_HISTORY;
constexpr int kFroBlocks = 256;  // partial sums of ||A||_F^2

// Device-resident state of one refinement, laid out as tqr_refine_report.
typedef tqr_refine_report RefineState;

// One problem of a refinement: the caller's A and B, the iterate X (n x
// nrhs), the residual R (m x nrhs), A^T R and then the correction S (n x
// nrhs; null for classical refinement, whose correction overwrites R in
// place), scratch of refine_partial_bytes, the state and an optional info
// word.  `square` selects the stopping measure (Rigal-Gaches for square
// systems, Stewart's bound otherwise), independently of where the
// correction comes from.
struct RefProb {
  const double *A;
  int64_t lda, m, n;
  const double *B;
  int64_t ldb, nrhs;
  double *X;
  int64_t ldx;
  double *R;
  int64_t ldr;
  double *S;
  int64_t lds;
  void *partial;
  RefineState *st;
  int32_t *info;
  int32_t square;
  int32_t pad_;
};

struct CopyDesc {
  const double *src;
  int64_t lds;
  double *dst;
  int64_t ldd;
  int64_t rows, cols;
};

size_t refine_partial_bytes(int64_t m, int64_t n, int64_t nrhs);
// `tab` null: the single problem `one` (count 1); else a device table of
// `count` problems with largest sizes mmax x nmax.
hipError_t refine_start(const RefProb *tab, const RefProb &one, int count, hipStream_t s);
hipError_t refine_fro(const RefProb *tab, const RefProb &one, int count, hipStream_t s);
hipError_t refine_residual(const RefProb *tab, const RefProb &one, int count, int64_t mmax, int64_t nmax,
                           hipStream_t s);
hipError_t refine_check(const RefProb *tab, const RefProb &one, int count, double tol, int it, hipStream_t s);
hipError_t refine_update(const RefProb *tab, const RefProb &one, int count, int64_t nmax, int64_t nrhs,
                         hipStream_t s);
hipError_t refine_finish(const RefProb *tab, const RefProb &one, int count, int32_t noconv, hipStream_t s);
hipError_t copy_batch(const CopyDesc *tab, int count, int64_t max_elems, hipStream_t s);

}  // namespace tqr
