// FP64 kernels of the least-squares refinement that follows a factorization
// with low-precision updates: residuals r = b - A x and s = A^T r with
// compensated dot products, the stopping test on the normwise backward
// error, and the correction x += d.  Every kernel first reads the
// refinement's `done` flag and returns at once when it is set, so that a
// fixed number of iterations can be enqueued without host round trips.
//
// Each kernel serves one problem (passed by value) or a batch (a device
// table, one problem per blockIdx.z).
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

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

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

__device__ __forceinline__ const RefProb &pick(const RefProb *tab, const RefProb &one) {
  return tab ? tab[blockIdx.z] : one;
}

__device__ __forceinline__ double *fro_of(const RefProb &P) { return static_cast<double *>(P.partial); }
__device__ __forceinline__ dd *part_of(const RefProb &P) {
  return reinterpret_cast<dd *>(static_cast<char *>(P.partial) + (size_t)kFroBlocks * sizeof(double));
}

// partial[(z * nch + y) * m + i] = sum over columns j of chunk y of A(i, j) X(j, z)
__global__ __launch_bounds__(RT) void resid_partial(const RefProb *tab, RefProb one) {
  const RefProb &P = pick(tab, one);
  if (P.st->done) return;
  const int64_t nch = (P.n + RCHUNK - 1) / RCHUNK;
  const int64_t y = blockIdx.y;
  if (y >= nch || (int64_t)blockIdx.x * RT >= P.m) return;
  const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
  const int64_t j0 = y * RCHUNK, j1 = min(P.n, j0 + RCHUNK);
  __shared__ double xs[RCHUNK];
  for (int64_t z = 0; z < P.nrhs; z++) {
    __syncthreads();
    for (int64_t j = j0 + threadIdx.x; j < j1; j += RT) xs[j - j0] = P.X[z * P.ldx + j];
    __syncthreads();
    if (i < P.m) {
      dd acc{0.0, 0.0};
      for (int64_t j = j0; j < j1; j++) dot2_step(acc, P.A[j * P.lda + i], xs[j - j0]);
      part_of(P)[(z * nch + y) * P.m + i] = acc;
    }
  }
}

// R(i, z) = B(i, z) - sum_y partial  (compensated over the chunks)
__global__ __launch_bounds__(RT) void resid_reduce(const RefProb *tab, RefProb one) {
  const RefProb &P = pick(tab, one);
  if (P.st->done) return;
  const int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (i >= P.m) return;
  const int64_t nch = (P.n + RCHUNK - 1) / RCHUNK;
  const dd *part = part_of(P);
  for (int64_t z = 0; z < P.nrhs; z++) {
    dd acc{P.B[z * P.ldb + i], 0.0};
    for (int64_t y = 0; y < nch; y++) {
      const dd p = part[(z * nch + y) * P.m + i];
      acc = dd_add(acc, dd{-p.hi, -p.lo});
    }
    P.R[z * P.ldr + i] = acc.hi + acc.lo;
  }
}

// S(j, z) = sum_i A(i, j) R(i, z): one wave per column j
__global__ __launch_bounds__(RT) void atr(const RefProb *tab, RefProb one) {
  const RefProb &P = pick(tab, one);
  if (P.st->done || !P.S) return;
  const int64_t j = (int64_t)blockIdx.x * (RT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= P.n) return;  // whole waves leave together
  for (int64_t z = 0; z < P.nrhs; z++) {
    dd acc{0.0, 0.0};
    for (int64_t i = lane; i < P.m; i += 64) dot2_step(acc, P.A[j * P.lda + i], P.R[z * P.ldr + i]);
    acc = wave_sum_dd(acc);
    if (lane == 0) P.S[z * P.lds + j] = acc.hi + acc.lo;
  }
}

// Squares of A's entries, per block of columns, for ||A||_F.
__global__ __launch_bounds__(RT) void fro_partial(const RefProb *tab, RefProb one) {
  const RefProb &P = pick(tab, one);
  __shared__ double red[RT / 64];
  double s = 0.0;
  for (int64_t j = blockIdx.x; j < P.n; j += gridDim.x)
    for (int64_t i = threadIdx.x; i < P.m; i += RT) {
      const double v = P.A[j * P.lda + i];
      s = fma(v, v, s);
    }
  s = block_sum(s, red);
  if (threadIdx.x == 0) fro_of(P)[blockIdx.x] = s;
}

// Stopping test of iteration `it`.  Square problems: normwise backward
// error ||r|| / (||A||_F ||x|| + ||b||) (Rigal and Gaches); rectangular
// ones: ||A^T r|| / (||A||_F ||r||), Stewart's bound on the backward error
// of a least-squares solution.  The test passes when every right-hand side
// meets tol; `done` then stops every later kernel of this problem.
__global__ __launch_bounds__(RT) void check(const RefProb *tab, RefProb one, double tol, int it) {
  const RefProb &P = pick(tab, one);
  if (P.st->done) return;
  __shared__ double red[RT / 64];
  double f = 0.0;
  for (int i = threadIdx.x; i < kFroBlocks; i += RT) f += fro_of(P)[i];
  const double anorm = sqrt(block_sum(f, red));
  double worst = 0.0;
  for (int64_t z = 0; z < P.nrhs; z++) {
    double rr = 0.0;
    for (int64_t i = threadIdx.x; i < P.m; i += RT) rr = fma(P.R[z * P.ldr + i], P.R[z * P.ldr + i], rr);
    const double rn = sqrt(block_sum(rr, red));
    double be;
    if (P.square) {
      double xx = 0.0, bb = 0.0;
      for (int64_t i = threadIdx.x; i < P.n; i += RT) xx = fma(P.X[z * P.ldx + i], P.X[z * P.ldx + i], xx);
      for (int64_t i = threadIdx.x; i < P.m; i += RT) bb = fma(P.B[z * P.ldb + i], P.B[z * P.ldb + i], bb);
      const double xn = sqrt(block_sum(xx, red)), bn = sqrt(block_sum(bb, red));
      be = rn / (anorm * xn + bn);
    } else {
      double ss = 0.0;
      for (int64_t i = threadIdx.x; i < P.n; i += RT) ss = fma(P.S[z * P.lds + i], P.S[z * P.lds + i], ss);
      const double sn = sqrt(block_sum(ss, red));
      be = (rn == 0.0) ? 0.0 : sn / (anorm * rn);
    }
    // a NaN or infinite measure (overflow in the low-precision updates, a
    // non-finite input) is a failure, never a pass: fmax would drop a NaN
    if (!(be <= 1.7976931348623157e308)) be = INFINITY;
    worst = fmax(worst, be);
  }
  if (threadIdx.x == 0) {
    P.st->backward_error = worst;
    if (it < kRefineHistory) P.st->history[it] = worst;
    P.st->iterations = it;
    if (worst <= tol) P.st->done = 1;
  }
}

// X += D: D = S when the correction came from the semi-normal equations
// (S given), else the first n rows of R (classical refinement, in place).
__global__ __launch_bounds__(RT) void update(const RefProb *tab, RefProb one) {
  const RefProb &P = pick(tab, one);
  if (P.st->done) return;
  const int64_t k = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (k >= P.n * P.nrhs) return;
  const int64_t z = k / P.n, i = k % P.n;
  const double d = P.S ? P.S[z * P.lds + i] : P.R[z * P.ldr + i];
  P.X[z * P.ldx + i] += d;
}

__global__ void start(const RefProb *tab, RefProb one, int count) {
  for (int x = threadIdx.x; x < count; x += blockDim.x) {
    const RefProb &P = tab ? tab[x] : one;
    P.st->done = 0;
    P.st->iterations = 0;
    P.st->backward_error = -1.0;
    for (int i = 0; i < kRefineHistory; i++) P.st->history[i] = -1.0;
    P.st->gmres_steps = 0;
    P.st->krylov_steps = 0;
  }
}

__global__ void finish(const RefProb *tab, RefProb one, int count, int32_t noconv) {
  for (int x = threadIdx.x; x < count; x += blockDim.x) {
    const RefProb &P = tab ? tab[x] : one;
    if (P.info && !P.st->done && *P.info == 0) *P.info = noconv;
  }
}

// Column-major block copies, one per blockIdx.z.
__global__ __launch_bounds__(RT) void copy_blocks(const CopyDesc *tab) {
  const CopyDesc &c = tab[blockIdx.z];
  const int64_t tot = c.rows * c.cols;
  for (int64_t k = (int64_t)blockIdx.x * RT + threadIdx.x; k < tot; k += (int64_t)gridDim.x * RT) {
    const int64_t j = k / c.rows, i = k % c.rows;
    c.dst[j * c.ldd + i] = c.src[j * c.lds + i];
  }
}

dim3 grid3(int64_t x, int64_t y, int64_t z) { return dim3((unsigned)(x < 1 ? 1 : x), (unsigned)(y < 1 ? 1 : y), (unsigned)z); }

}  // namespace

size_t refine_partial_bytes(int64_t m, int64_t n, int64_t nrhs) {
  const int64_t nch = (n + RCHUNK - 1) / RCHUNK;
  return (size_t)kFroBlocks * sizeof(double) + (size_t)(nch * m * nrhs) * sizeof(dd);
}

// Launch helpers: `tab` null means the single problem `one`; otherwise
// `count` problems whose largest sizes are mmax, nmax.
hipError_t refine_start(const RefProb *tab, const RefProb &one, int count, hipStream_t s) {
  hipLaunchKernelGGL(start, dim3(1), dim3(RT), 0, s, tab, one, count);
  return hipGetLastError();
}

hipError_t refine_fro(const RefProb *tab, const RefProb &one, int count, hipStream_t s) {
  hipLaunchKernelGGL(fro_partial, grid3(kFroBlocks, 1, count), dim3(RT), 0, s, tab, one);
  return hipGetLastError();
}

hipError_t refine_residual(const RefProb *tab, const RefProb &one, int count, int64_t mmax, int64_t nmax,
                           hipStream_t s) {
  const int64_t nch = (nmax + RCHUNK - 1) / RCHUNK;
  const int64_t rb = (mmax + RT - 1) / RT;
  hipLaunchKernelGGL(resid_partial, grid3(rb, nch, count), dim3(RT), 0, s, tab, one);
  hipLaunchKernelGGL(resid_reduce, grid3(rb, 1, count), dim3(RT), 0, s, tab, one);
  hipLaunchKernelGGL(atr, grid3((nmax + RT / 64 - 1) / (RT / 64), 1, count), dim3(RT), 0, s, tab, one);
  return hipGetLastError();
}

hipError_t refine_check(const RefProb *tab, const RefProb &one, int count, double tol, int it, hipStream_t s) {
  hipLaunchKernelGGL(check, grid3(1, 1, count), dim3(RT), 0, s, tab, one, tol, it);
  return hipGetLastError();
}

hipError_t refine_update(const RefProb *tab, const RefProb &one, int count, int64_t nmax, int64_t nrhs,
                         hipStream_t s) {
  hipLaunchKernelGGL(update, grid3((nmax * nrhs + RT - 1) / RT, 1, count), dim3(RT), 0, s, tab, one);
  return hipGetLastError();
}

hipError_t refine_finish(const RefProb *tab, const RefProb &one, int count, int32_t noconv, hipStream_t s) {
  hipLaunchKernelGGL(finish, dim3(1), dim3(RT), 0, s, tab, one, count, noconv);
  return hipGetLastError();
}

hipError_t copy_batch(const CopyDesc *tab, int count, int64_t max_elems, hipStream_t s) {
  int64_t blocks = (max_elems + RT - 1) / RT;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(copy_blocks, grid3(blocks, 1, count), dim3(RT), 0, s, tab);
  return hipGetLastError();
}

}  // namespace tqr
