// FP64 kernels of the least-squares refinement that follows a factorization
// with low-precision updates: residuals r = b - A x and s = A^T r with
// compensated dot products, the stopping test on the normwise backward
// error, and the correction x += d.  Every kernel first reads the
// refinement's `done` flag and returns at once when it is set, so that a
// fixed number of iterations can be enqueued without host round trips.
//
// Compensated dot product (Ogita, Rump and Oishi, "Accurate sum and dot
// product", SIAM J. Sci. Comput. 26, 2005, algorithm Dot2): each product is
// split exactly with an FMA (a*b = p + e), each sum exactly with Knuth's
// TwoSum, and the error terms are accumulated separately; the result is as
// accurate as if computed in twice the working precision and then rounded.
// These kernels stream A from HBM once per call, so the extra arithmetic is
// free.
#include <hip/hip_runtime.h>

#include "refine.h"

namespace tqr {

namespace {

constexpr int RT = 256;      // threads per block
constexpr int RCHUNK = 256;  // columns of A per residual partial sum

struct dd {
  double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double z = s - a;
  e = (a - (s - z)) + (b - z);
}

// acc += a * b, compensated
__device__ __forceinline__ void dot2_step(dd &acc, double a, double b) {
  const double p = a * b;
  const double pe = fma(a, b, -p);
  double s, se;
  two_sum(acc.hi, p, s, se);
  acc.hi = s;
  acc.lo += pe + se;
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
  double s, e;
  two_sum(x.hi, y.hi, s, e);
  return dd{s, e + x.lo + y.lo};
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, 64);
}

__device__ __forceinline__ dd wave_sum_dd(dd v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    dd o{shfl_xor_d(v.hi, m), shfl_xor_d(v.lo, m)};
    v = dd_add(v, o);
  }
  return v;
}

// Sum over a block of RT threads (every thread receives the result).
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < RT / 64; i++) t += red[i];
  return t;
}

// partial[(z * nch + y) * m + i] = sum over columns j of chunk y of A(i, j) x(j, z)
__global__ __launch_bounds__(RT) void resid_partial(const double *A, int64_t lda, int64_t m, int64_t n,
                                                    const double *X, int64_t ldx, dd *partial,
                                                    const RefineState *st) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
  const int64_t y = blockIdx.y, z = blockIdx.z;
  const int64_t nch = gridDim.y;
  const int64_t j0 = y * RCHUNK, j1 = min(n, j0 + RCHUNK);
  __shared__ double xs[RCHUNK];
  for (int64_t j = j0 + threadIdx.x; j < j1; j += RT) xs[j - j0] = X[z * ldx + j];
  __syncthreads();
  if (i >= m) return;
  dd acc{0.0, 0.0};
  for (int64_t j = j0; j < j1; j++) dot2_step(acc, A[j * lda + i], xs[j - j0]);
  partial[(z * nch + y) * m + i] = acc;
}

// R(i, z) = B(i, z) - sum_y partial  (compensated over the chunks)
__global__ __launch_bounds__(RT) void resid_reduce(int64_t m, int nch, const dd *partial, const double *B,
                                                   int64_t ldb, double *R, int64_t ldr,
                                                   const RefineState *st) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
  const int64_t z = blockIdx.y;
  if (i >= m) return;
  dd acc{B[z * ldb + i], 0.0};
  for (int y = 0; y < nch; y++) {
    const dd p = partial[(z * nch + y) * m + i];
    acc = dd_add(acc, dd{-p.hi, -p.lo});
  }
  R[z * ldr + i] = acc.hi + acc.lo;
}

// S(j, z) = sum_i A(i, j) R(i, z): one wave per (column j, right-hand side z)
__global__ __launch_bounds__(RT) void atr(const double *A, int64_t lda, int64_t m, int64_t n,
                                          const double *R, int64_t ldr, double *S, int64_t lds,
                                          const RefineState *st) {
  if (st->done) return;
  const int64_t j = (int64_t)blockIdx.x * (RT / 64) + (threadIdx.x >> 6);
  const int64_t z = blockIdx.y;
  const int lane = threadIdx.x & 63;
  if (j >= n) return;  // whole waves leave together
  dd acc{0.0, 0.0};
  for (int64_t i = lane; i < m; i += 64) dot2_step(acc, A[j * lda + i], R[z * ldr + i]);
  acc = wave_sum_dd(acc);
  if (lane == 0) S[z * lds + j] = acc.hi + acc.lo;
}

// Squares of A's entries, per block of columns, for ||A||_F.
__global__ __launch_bounds__(RT) void fro_partial(const double *A, int64_t lda, int64_t m, int64_t n,
                                                  double *out) {
  __shared__ double red[RT / 64];
  double s = 0.0;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
    for (int64_t i = threadIdx.x; i < m; i += RT) {
      const double v = A[j * lda + i];
      s = fma(v, v, s);
    }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Stopping test of iteration `it`.  Square problems: normwise backward
// error ||r|| / (||A||_F ||x|| + ||b||) (Rigal and Gaches); rectangular
// ones: ||A^T r|| / (||A||_F ||r||), Stewart's bound on the backward error
// of a least-squares solution.  The test passes when every right-hand side
// meets tol; `done` then stops every later kernel.
__global__ __launch_bounds__(RT) void check(int64_t m, int64_t n, int64_t nrhs, const double *R, int64_t ldr,
                                            const double *S, int64_t lds, const double *X, int64_t ldx,
                                            const double *B, int64_t ldb, const double *fro, int nfro,
                                            double tol, int square, int it, RefineState *st) {
  if (st->done) return;
  __shared__ double red[RT / 64];
  double f = 0.0;
  for (int i = threadIdx.x; i < nfro; i += RT) f += fro[i];
  const double anorm = sqrt(block_sum(f, red));
  double worst = 0.0;
  for (int64_t z = 0; z < nrhs; z++) {
    double rr = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += RT) rr = fma(R[z * ldr + i], R[z * ldr + i], rr);
    const double rn = sqrt(block_sum(rr, red));
    double be;
    if (square) {
      double xx = 0.0, bb = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += RT) xx = fma(X[z * ldx + i], X[z * ldx + i], xx);
      for (int64_t i = threadIdx.x; i < m; i += RT) bb = fma(B[z * ldb + i], B[z * ldb + i], bb);
      const double xn = sqrt(block_sum(xx, red)), bn = sqrt(block_sum(bb, red));
      be = rn / (anorm * xn + bn);
    } else {
      double ss = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += RT) ss = fma(S[z * lds + i], S[z * lds + i], ss);
      const double sn = sqrt(block_sum(ss, red));
      be = (rn == 0.0) ? 0.0 : sn / (anorm * rn);
    }
    worst = fmax(worst, be);
  }
  if (threadIdx.x == 0) {
    st->backward_error = worst;
    if (it < kRefineHistory) st->history[it] = worst;
    st->iterations = it;
    if (worst <= tol) st->done = 1;
  }
}

// X += D
__global__ __launch_bounds__(RT) void update(int64_t n, int64_t nrhs, double *X, int64_t ldx, const double *D,
                                             int64_t ldd, const RefineState *st) {
  if (st->done) return;
  const int64_t k = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (k >= n * nrhs) return;
  const int64_t z = k / n, i = k % n;
  X[z * ldx + i] += D[z * ldd + i];
}

__global__ void start(RefineState *st) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->iterations = 0;
    st->backward_error = -1.0;
    for (int i = 0; i < kRefineHistory; i++) st->history[i] = -1.0;
  }
}

__global__ void finish(const RefineState *st, int32_t *info, int32_t noconv) {
  if (threadIdx.x == 0 && info && !st->done && *info == 0) *info = noconv;
}

}  // namespace

// Scratch layout: kFroBlocks doubles (column-block sums of squares of A),
// then the residual partial sums (chunks x m x nrhs compensated pairs).
size_t refine_partial_bytes(int64_t m, int64_t n, int64_t nrhs) {
  const int64_t nch = (n + RCHUNK - 1) / RCHUNK;
  return (size_t)kFroBlocks * sizeof(double) + (size_t)(nch * m * nrhs) * sizeof(dd);
}

hipError_t refine_start(RefineState *st, hipStream_t s) {
  hipLaunchKernelGGL(start, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t refine_fro(const double *A, int64_t lda, int64_t m, int64_t n, void *partial, hipStream_t s) {
  double *fro = static_cast<double *>(partial);
  hipLaunchKernelGGL(fro_partial, dim3(kFroBlocks), dim3(RT), 0, s, A, lda, m, n, fro);
  return hipGetLastError();
}

hipError_t refine_residual(const double *A, int64_t lda, int64_t m, int64_t n, const double *X, int64_t ldx,
                           const double *B, int64_t ldb, int64_t nrhs, double *R, int64_t ldr, double *S,
                           int64_t lds, void *partial, const RefineState *st, hipStream_t s) {
  const int nch = (int)((n + RCHUNK - 1) / RCHUNK);
  dd *p = reinterpret_cast<dd *>(static_cast<char *>(partial) + (size_t)kFroBlocks * sizeof(double));
  const unsigned rb = (unsigned)((m + RT - 1) / RT);
  hipLaunchKernelGGL(resid_partial, dim3(rb, nch, (unsigned)nrhs), dim3(RT), 0, s, A, lda, m, n, X, ldx, p, st);
  hipLaunchKernelGGL(resid_reduce, dim3(rb, (unsigned)nrhs), dim3(RT), 0, s, m, nch, p, B, ldb, R, ldr, st);
  if (S)
    hipLaunchKernelGGL(atr, dim3((unsigned)((n + RT / 64 - 1) / (RT / 64)), (unsigned)nrhs), dim3(RT), 0, s, A,
                       lda, m, n, R, ldr, S, lds, st);
  return hipGetLastError();
}

hipError_t refine_check(int64_t m, int64_t n, int64_t nrhs, const double *R, int64_t ldr, const double *S,
                        int64_t lds, const double *X, int64_t ldx, const double *B, int64_t ldb,
                        const void *partial, double tol, int it, RefineState *st, hipStream_t s) {
  const double *fro = static_cast<const double *>(partial);
  hipLaunchKernelGGL(check, dim3(1), dim3(RT), 0, s, m, n, nrhs, R, ldr, S, lds, X, ldx, B, ldb, fro,
                     kFroBlocks, tol, S ? 0 : 1, it, st);
  return hipGetLastError();
}

hipError_t refine_update(int64_t n, int64_t nrhs, double *X, int64_t ldx, const double *D, int64_t ldd,
                         const RefineState *st, hipStream_t s) {
  const int64_t tot = n * nrhs;
  hipLaunchKernelGGL(update, dim3((unsigned)((tot + RT - 1) / RT)), dim3(RT), 0, s, n, nrhs, X, ldx, D, ldd, st);
  return hipGetLastError();
}

hipError_t refine_finish(const RefineState *st, int32_t *info, int32_t noconv, hipStream_t s) {
  hipLaunchKernelGGL(finish, dim3(1), dim3(64), 0, s, st, info, noconv);
  return hipGetLastError();
}

}  // namespace tqr
