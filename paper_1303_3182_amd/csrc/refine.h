// Refinement kernels (refine.hip): FP64 residuals with compensated dot
// products, the backward-error stopping test and the correction update.
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

size_t refine_partial_bytes(int64_t m, int64_t n, int64_t nrhs);
hipError_t refine_start(RefineState *st, hipStream_t s);
hipError_t refine_fro(const double *A, int64_t lda, int64_t m, int64_t n, void *partial, hipStream_t s);
// R = B - A X (m x nrhs); if S is not null, also S = A^T R (n x nrhs).
hipError_t refine_residual(const double *A, int64_t lda, int64_t m, int64_t n, const double *X, int64_t ldx,
                           const double *B, int64_t ldb, int64_t nrhs, double *R, int64_t ldr, double *S,
                           int64_t lds, void *partial, const RefineState *st, hipStream_t s);
// Backward error of the current X (square when S is null); sets done when <= tol.
hipError_t refine_check(int64_t m, int64_t n, int64_t nrhs, const double *R, int64_t ldr, const double *S,
                        int64_t lds, const double *X, int64_t ldx, const double *B, int64_t ldb,
                        const void *partial, double tol, int it, RefineState *st, hipStream_t s);
hipError_t refine_update(int64_t n, int64_t nrhs, double *X, int64_t ldx, const double *D, int64_t ldd,
                         const RefineState *st, hipStream_t s);
hipError_t refine_finish(const RefineState *st, int32_t *info, int32_t noconv, hipStream_t s);

}  // namespace tqr
