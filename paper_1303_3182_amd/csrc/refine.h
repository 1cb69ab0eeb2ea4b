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

// ------------------------------------------------ GMRES refinement (gmres.hip)
constexpr int kGmresMax = 64;  // Krylov directions per outer step, at most

// Device state of the GMRES cycle of one square problem.
struct GmState {
  int32_t j;            // directions built in the current cycle
  int32_t inner_done;   // the cycle has converged (or reached its limit)
  double beta;          // ||M^{-1} r|| at the cycle's start
  double resid;         // preconditioned residual estimate |g(j)|
};

struct GmArgs {
  const double *A;  // the caller's FP64 matrix (n x n, lda)
  int64_t lda, n;
  double *V;        // n x (kmax + 1) Krylov basis
  double *H;        // (kmax + 1) x kmax Hessenberg matrix, column-major
  double *cs, *sn, *gv;  // Givens rotations and the rotated right-hand side
  double *x;        // iterate (n)
  double *z;        // work vector: operand of M^{-1} (length >= n)
  double *part;     // matrix-vector partial sums (gmres_partial_bytes)
  GmState *st;
  RefineState *rep;  // the refinement's report: every kernel returns once rep->done
                     // is set; rep->gmres_steps / krylov_steps count the work
  double tol;       // relative reduction of the preconditioned residual per cycle
  int32_t kmax;
  int32_t pad_;
};

size_t gmres_bytes(int64_t n, int kmax);
size_t gmres_partial_bytes(int64_t n);
GmArgs gmres_args(void *mem, int64_t n, int kmax, const double *A, int64_t lda, double *x, double *z,
                  void *partial, RefineState *rep, double tol);
// a cycle: gmres_init (z = M^{-1} r given), then per step j: z = A v_j
// (gmres_matvec), z <- M^{-1} z (the executor), gmres_arnoldi; then
// gmres_update (x += V y)
hipError_t gmres_init(const GmArgs &g, hipStream_t s);
hipError_t gmres_matvec(const GmArgs &g, int j, hipStream_t s);
hipError_t gmres_arnoldi(const GmArgs &g, int j, hipStream_t s);
hipError_t gmres_update(const GmArgs &g, hipStream_t s);

}  // namespace tqr
