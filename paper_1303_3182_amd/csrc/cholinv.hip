// Tile kernels of the tile Cholesky inversion (thesis chapter "Cholesky
// Inversion", algorithm alg:InPlace) and the persistent executor that runs
// its task graph.  FP64, gfx950, NB x NB tiles of a column-major matrix.
//
// Every task stages its operand tiles in LDS (column-major, padded stride),
// computes there or in registers, and writes its result tile: all global
// reads of a task precede its writes, so a task whose output aliases an
// input (the in-place TRMMs, LAUUM) needs no other care.  Only the lower
// triangle of the matrix is read or written.  Tiles past n are padded: zero
// off the diagonal, one on the diagonal of a diagonal tile (so the Cholesky
// factor and the inverse of a padded diagonal tile are padded with the
// identity); stores skip the padding.
//
// Products C = beta Z + alpha op(X) op(Y): each thread holds an RB x RB
// block of C in registers (rows tr + 16a, columns tc + 16b), reading X and
// Y from LDS; on this chip FP64 FMA runs at the FP64 matrix rate, so the
// plain FMA formulation loses nothing to the matrix cores.
#include <hip/hip_runtime.h>

#include "exec_loop.h"
#include "tqr_types.h"

namespace tqr {

namespace {

constexpr int CT = 256;  // threads per workgroup

template <int NB>
struct CholSmem {
  static constexpr int LD = NB + 1;
  double X[NB * LD];
  double Y[NB * LD];
  double Z[NB * LD];
  int task;
};

enum LoadMode { LD_FULL = 0, LD_LOWER = 1, LD_DIAG = 2 };

// dst = tile (rows x cols valid) of src; LD_LOWER zeroes the strict upper
// triangle; LD_DIAG also puts ones on the padded part of the diagonal.
// Every load of the thread is issued before its first LDS store (clamped
// addresses, masked values), so the tile costs one memory latency rather
// than one per element.
template <int NB>
__device__ __forceinline__ void load_tile(const double *__restrict__ src, int64_t ld, int rows, int cols,
                                          double *dst, int mode) {
  constexpr int LD = CholSmem<NB>::LD;
  constexpr int PER = NB * NB / CT;
  static_assert(PER * CT == NB * NB, "a tile splits evenly over the threads");
  double v[PER];
#pragma unroll
  for (int it = 0; it < PER; it++) {
    const int idx = threadIdx.x + it * CT;
    const int r = idx % NB, c = idx / NB;
    const bool in = r < rows && c < cols && (mode == LD_FULL || r >= c);
    const double x = src[(int64_t)(in ? c : 0) * ld + (in ? r : 0)];
    v[it] = in ? x : 0.0;
  }
#pragma unroll
  for (int it = 0; it < PER; it++) {
    const int idx = threadIdx.x + it * CT;
    const int r = idx % NB, c = idx / NB;
    double x = v[it];
    if (mode == LD_DIAG && r == c && (r >= rows || c >= cols)) x = 1.0;
    dst[c * LD + r] = x;
  }
}

template <int NB>
__device__ __forceinline__ void store_tile(double *__restrict__ dst, int64_t ld, int rows, int cols,
                                           const double *src, bool lower) {
  constexpr int LD = CholSmem<NB>::LD;
  for (int idx = threadIdx.x; idx < NB * NB; idx += CT) {
    const int r = idx % NB, c = idx / NB;
    if (r < rows && c < cols && (!lower || r >= c)) dst[(int64_t)c * ld + r] = src[c * LD + r];
  }
}

// C = beta Z + alpha op(X) op(Y) (op = transpose when TX / TY), written to
// dst (rows x cols valid; lower triangle only when `lower`), and to copy
// when given.  X, Y, Z are in LDS.
template <int NB, bool TX, bool TY>
__device__ __forceinline__ void product(const CholSmem<NB> &sm, double alpha, double beta, double *dst,
                                        int64_t ld, int rows, int cols, bool lower, double *copy,
                                        int64_t ldc) {
  constexpr int LD = CholSmem<NB>::LD;
  constexpr int RB = NB / 16;
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  double acc[RB][RB];
#pragma unroll
  for (int a = 0; a < RB; a++)
#pragma unroll
    for (int b = 0; b < RB; b++) acc[a][b] = 0.0;
#pragma unroll 4
  for (int k = 0; k < NB; k++) {
    double xv[RB], yv[RB];
#pragma unroll
    for (int a = 0; a < RB; a++) {
      const int r = tr + 16 * a;
      xv[a] = TX ? sm.X[r * LD + k] : sm.X[k * LD + r];
    }
#pragma unroll
    for (int b = 0; b < RB; b++) {
      const int c = tc + 16 * b;
      yv[b] = TY ? sm.Y[k * LD + c] : sm.Y[c * LD + k];
    }
#pragma unroll
    for (int a = 0; a < RB; a++)
#pragma unroll
      for (int b = 0; b < RB; b++) acc[a][b] = fma(xv[a], yv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < RB; a++)
#pragma unroll
    for (int b = 0; b < RB; b++) {
      const int r = tr + 16 * a, c = tc + 16 * b;
      const double v = (beta != 0.0 ? beta * sm.Z[c * LD + r] : 0.0) + alpha * acc[a][b];
      if (r < rows && c < cols && (!lower || r >= c)) {
        dst[(int64_t)c * ld + r] = v;
        if (copy) copy[(int64_t)c * ldc + r] = v;
      }
    }
}

// The three diagonal-tile kernels (Cholesky factor, triangular solve,
// triangular inverse) run in one wave, lane r holding row r of the tile in
// registers (loops unrolled, so the row is a register array): the factor's
// columns are broadcast with readlane, a static triangle with LDS broadcast
// reads.  No workgroup barrier inside; each performs the same operations in
// the same order as the column-by-column formulation in its comment.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky factor of the tile in Z (lower, in place), right-looking: for
// each column c, L(c,c) = sqrt(A(c,c)), L(r,c) = A(r,c) / L(c,c) (r > c),
// A(r,s) -= L(r,c) L(s,c) (r >= s > c).  A non-positive (or NaN) pivot
// records the 1-based global index base + c + 1 of the first such column
// in *notpd.
template <int NB>
__device__ __forceinline__ void potrf_lds(CholSmem<NB> &sm, int base, int32_t *notpd) {
  constexpr int LD = CholSmem<NB>::LD;
  __syncthreads();  // the tile is in Z
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    const int rr = r < NB ? r : 0;  // lanes past the tile read row 0 and write nothing
    double a[NB];
#pragma unroll
    for (int s = 0; s < NB; s++) a[s] = sm.Z[s * LD + rr];
#pragma unroll
    for (int c = 0; c < NB; c++) {
      const double d = readlane_d(a[c], c);
      const bool ok = d > 0.0;
      const double piv = ok ? sqrt(d) : __builtin_nan("");
      if (!ok && r == 0) atomicMin(notpd, base + c + 1);
      a[c] = (r > c) ? a[c] / piv : (r == c ? piv : a[c]);
#pragma unroll
      for (int s = c + 1; s < NB; s++) {
        const double lsc = readlane_d(a[c], s);
        if (r >= s) a[s] = fma(-a[c], lsc, a[s]);
      }
    }
    if (r < NB) {
#pragma unroll
      for (int s = 0; s < NB; s++) sm.Z[s * LD + r] = a[s];
    }
  }
  __syncthreads();
}

// Z <- Z L^{-T} with L (lower) in X, row by row: for each column c,
// Z(r,c) /= L(c,c), then Z(r,s) -= Z(r,c) L(s,c) for s > c.
template <int NB>
__device__ __forceinline__ void trsm_lds(CholSmem<NB> &sm) {
  constexpr int LD = CholSmem<NB>::LD;
  const double *L = sm.X;
  __syncthreads();  // X and Z are loaded
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    const int rr = r < NB ? r : 0;
    double z[NB];
#pragma unroll
    for (int s = 0; s < NB; s++) z[s] = sm.Z[s * LD + rr];
#pragma unroll
    for (int c = 0; c < NB; c++) {
      z[c] /= L[c * LD + c];
#pragma unroll
      for (int s = c + 1; s < NB; s++) z[s] = fma(-z[c], L[c * LD + s], z[s]);
    }
    if (r < NB) {
#pragma unroll
      for (int s = 0; s < NB; s++) sm.Z[s * LD + r] = z[s];
    }
  }
  __syncthreads();
}

// Z <- L^{-1} for L (lower) in Z, in place, from the last column: W(c,c) =
// 1/L(c,c), W(r,c) = -(sum_{c<k<=r} W(r,k) L(k,c)) W(c,c), r > c.  Row r of
// W stays in registers until every column is done, so L is read intact.
template <int NB>
__device__ __forceinline__ void trtri_lds(CholSmem<NB> &sm) {
  constexpr int LD = CholSmem<NB>::LD;
  __syncthreads();  // the tile is in Z
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    const int rr = r < NB ? r : 0;
    double w[NB];
#pragma unroll
    for (int c = 0; c < NB; c++) w[c] = sm.Z[c * LD + rr];  // L's upper part (r < c) is kept
#pragma unroll
    for (int c = NB - 1; c >= 0; c--) {
      const double wcc = 1.0 / sm.Z[c * LD + c];
      double v = 0.0;
#pragma unroll
      for (int k = c + 1; k < NB; k++)
        if (k <= r) v = fma(w[k], sm.Z[c * LD + k], v);
      v = -v * wcc;
      w[c] = (r > c) ? v : (r == c ? wcc : w[c]);
    }
    // (one wave: every lane's reads of L are done before these writes)
    if (r < NB) {
#pragma unroll
      for (int c = 0; c < NB; c++) sm.Z[c * LD + r] = w[c];
    }
  }
  __syncthreads();
}

template <int NB>
__device__ __forceinline__ void run_chol_task(const Problem &p, const Task &t, CholSmem<NB> &sm) {
  const int64_t lda = p.lda;
  const int64_t n = p.n;
  auto tile = [&](double *base, int64_t ld, int i, int j) { return base + (int64_t)j * NB * ld + (int64_t)i * NB; };
  auto dim = [&](int i) { return (int)min((int64_t)NB, n - (int64_t)i * NB); };
  // copies of L (end of step 1) and of L^{-1} (end of step 2), for the
  // variant with array renaming; null in place
  double *L0 = p.B, *W0 = p.Tf;
  const int64_t ldc = p.ldb;
  const int i = t.i, j = t.j, k = t.k;
  const int kind = t.kind;
  // source of a step-2 (step-3) read of tile (r, c): the copy when renamed
  auto src2 = [&](int r, int c) { return L0 ? tile(L0, ldc, r, c) : tile(p.A, lda, r, c); };
  auto src3 = [&](int r, int c) { return W0 ? tile(W0, ldc, r, c) : tile(p.A, lda, r, c); };
  auto ld2 = [&]() { return L0 ? ldc : lda; };
  auto ld3 = [&]() { return W0 ? ldc : lda; };
  switch (kind) {
    case K_POTRF: {  // A(j,j) <- chol(A(j,j))
      load_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.Z, LD_DIAG);
      __syncthreads();
      potrf_lds<NB>(sm, j * NB, p.singular);
      store_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.Z, true);
      if (L0) store_tile<NB>(tile(L0, ldc, j, j), ldc, dim(j), dim(j), sm.Z, true);
      break;
    }
    case K_CTRSM: {  // A(i,j) <- A(i,j) L(j,j)^{-T}
      load_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.X, LD_DIAG);
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Z, LD_FULL);
      __syncthreads();
      trsm_lds<NB>(sm);
      store_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Z, false);
      if (L0) store_tile<NB>(tile(L0, ldc, i, j), ldc, dim(i), dim(j), sm.Z, false);
      break;
    }
    case K_CSYRK: {  // A(j,j) <- A(j,j) - A(j,k) A(j,k)^T
      load_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.Z, LD_LOWER);
      load_tile<NB>(tile(p.A, lda, j, k), lda, dim(j), dim(k), sm.X, LD_FULL);
      load_tile<NB>(tile(p.A, lda, j, k), lda, dim(j), dim(k), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, false, true>(sm, -1.0, 1.0, tile(p.A, lda, j, j), lda, dim(j), dim(j), true, nullptr, 0);
      break;
    }
    case K_CGEMM: {  // A(i,j) <- A(i,j) - A(i,k) A(j,k)^T
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Z, LD_FULL);
      load_tile<NB>(tile(p.A, lda, i, k), lda, dim(i), dim(k), sm.X, LD_FULL);
      load_tile<NB>(tile(p.A, lda, j, k), lda, dim(j), dim(k), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, false, true>(sm, -1.0, 1.0, tile(p.A, lda, i, j), lda, dim(i), dim(j), false, nullptr, 0);
      break;
    }
    case K_TRTRI: {  // A(j,j) <- L(j,j)^{-1}
      load_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.Z, LD_DIAG);
      __syncthreads();
      trtri_lds<NB>(sm);
      store_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.Z, true);
      if (W0) store_tile<NB>(tile(W0, ldc, j, j), ldc, dim(j), dim(j), sm.Z, true);
      break;
    }
    case K_TRMML: {  // A(i,j) <- A(i,i) A(i,j), A(i,i) = L(i,i)^{-1}
      load_tile<NB>(tile(p.A, lda, i, i), lda, dim(i), dim(i), sm.X, LD_LOWER);
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, false, false>(sm, 1.0, 0.0, tile(p.A, lda, i, j), lda, dim(i), dim(j), false, nullptr, 0);
      break;
    }
    case K_IGEMM: {  // A(i,j) <- A(i,j) + A(i,k) L(k,j)
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Z, LD_FULL);
      load_tile<NB>(tile(p.A, lda, i, k), lda, dim(i), dim(k), sm.X, LD_FULL);
      load_tile<NB>(src2(k, j), ld2(), dim(k), dim(j), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, false, false>(sm, 1.0, 1.0, tile(p.A, lda, i, j), lda, dim(i), dim(j), false, nullptr, 0);
      break;
    }
    case K_TRMMR: {  // A(i,j) <- -A(i,j) A(j,j), A(j,j) = L(j,j)^{-1}
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.X, LD_FULL);
      load_tile<NB>(tile(p.A, lda, j, j), lda, dim(j), dim(j), sm.Y, LD_LOWER);
      __syncthreads();
      product<NB, false, false>(sm, -1.0, 0.0, tile(p.A, lda, i, j), lda, dim(i), dim(j), false,
                                W0 ? tile(W0, ldc, i, j) : nullptr, ldc);
      break;
    }
    case K_TRMMT: {  // A(i,j) <- W(i,i)^T A(i,j)
      load_tile<NB>(src3(i, i), ld3(), dim(i), dim(i), sm.X, LD_LOWER);
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, true, false>(sm, 1.0, 0.0, tile(p.A, lda, i, j), lda, dim(i), dim(j), false, nullptr, 0);
      break;
    }
    case K_LAUUM: {  // A(i,i) <- A(i,i)^T A(i,i), lower triangle
      load_tile<NB>(tile(p.A, lda, i, i), lda, dim(i), dim(i), sm.X, LD_LOWER);
      load_tile<NB>(tile(p.A, lda, i, i), lda, dim(i), dim(i), sm.Y, LD_LOWER);
      __syncthreads();
      product<NB, true, false>(sm, 1.0, 0.0, tile(p.A, lda, i, i), lda, dim(i), dim(i), true, nullptr, 0);
      break;
    }
    case K_PGEMM: {  // A(i,j) <- A(i,j) + W(k,i)^T W(k,j)
      load_tile<NB>(tile(p.A, lda, i, j), lda, dim(i), dim(j), sm.Z, LD_FULL);
      load_tile<NB>(src3(k, i), ld3(), dim(k), dim(i), sm.X, LD_FULL);
      load_tile<NB>(src3(k, j), ld3(), dim(k), dim(j), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, true, false>(sm, 1.0, 1.0, tile(p.A, lda, i, j), lda, dim(i), dim(j), false, nullptr, 0);
      break;
    }
    case K_PSYRK: {  // A(i,i) <- A(i,i) + W(k,i)^T W(k,i), lower triangle
      load_tile<NB>(tile(p.A, lda, i, i), lda, dim(i), dim(i), sm.Z, LD_LOWER);
      load_tile<NB>(src3(k, i), ld3(), dim(k), dim(i), sm.X, LD_FULL);
      load_tile<NB>(src3(k, i), ld3(), dim(k), dim(i), sm.Y, LD_FULL);
      __syncthreads();
      product<NB, true, false>(sm, 1.0, 1.0, tile(p.A, lda, i, i), lda, dim(i), dim(i), true, nullptr, 0);
      break;
    }
    default:
      break;
  }
}

template <int NB>
__global__ void chol_reset(ExecArgs a) {
  executor_reset(a);
}

template <int NB>
__global__ __launch_bounds__(CT, 1) void exec_cholinv(ExecArgs a) {
  __shared__ CholSmem<NB> sm;
  if (a.skip && *a.skip) return;
  executor_loop(a, &sm.task, [&](const Task &t) { run_chol_task<NB>(a.prob, t, sm); });
}

__global__ void chol_finish(ExecArgs a, int32_t *info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int e = a.ctl->error;
    const int z = *a.prob.singular;
    if (info) *info = (e != 0) ? e : (z != 0x7fffffff ? z : 0);
  }
}

template <int NB>
hipError_t launch_nb(const ExecArgs &a, int grid, int32_t *info, hipStream_t s) {
  const int rgrid = (int)((a.ntasks + 255) / 256);
  hipLaunchKernelGGL(chol_reset<NB>, dim3(rgrid < 1 ? 1 : (rgrid > 1024 ? 1024 : rgrid)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(exec_cholinv<NB>, dim3(grid), dim3(CT), 0, s, a);
  hipLaunchKernelGGL(chol_finish, dim3(1), dim3(64), 0, s, a, info);
  return hipGetLastError();
}

template <int NB>
int occupancy_nb() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, exec_cholinv<NB>, CT, 0) != hipSuccess) return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

bool cholinv_nb_supported(int nb) { return nb == 32 || nb == 64; }

int cholinv_occupancy(int nb) { return nb == 32 ? occupancy_nb<32>() : occupancy_nb<64>(); }

hipError_t launch_cholinv(const ExecArgs &a, int nb, int grid, int32_t *info, hipStream_t s) {
  if (nb == 32) return launch_nb<32>(a, grid, info, s);
  if (nb == 64) return launch_nb<64>(a, grid, info, s);
  return hipErrorInvalidValue;
}

}  // namespace tqr
