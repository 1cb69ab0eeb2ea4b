// FP64 GMRES kernels of the GMRES-based refinement of a square system whose
// factorization used low-precision updates (project addition; the thesis
// treats FP64 only).  Each outer step solves the correction equation
// A d = r with GMRES left-preconditioned by the computed factors,
// M^{-1} = R^{-1} Q^T (Carson and Higham, "Accelerating the solution of
// linear systems by iterative refinement in three precisions", SIAM J. Sci.
// Comput. 40, 2018): the preconditioned operator M^{-1} A stays well
// conditioned even when kappa(A) u_low exceeds one, where plain refinement
// stalls.  The library applies M^{-1} with its executor (Q^T and the
// back-substitution); these kernels do the matrix-vector product with the
// caller's FP64 A, the Arnoldi step (modified Gram-Schmidt, two sweeps for
// orthogonality to working precision), the Givens rotations of the
// Hessenberg least-squares problem, and the final x += V y.
#include <hip/hip_runtime.h>

#include "refine.h"

namespace tqr {

namespace {

constexpr int GT = 256;       // threads per block of the matrix-vector product
constexpr int GCHUNK = 256;   // columns per partial sum
constexpr int AT = 1024;      // threads of the one-block Arnoldi kernels

__device__ __forceinline__ double block_sum_1k(double v, double *red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += red[i];
  return t;
}

__device__ __forceinline__ bool stopped(const GmArgs &g) { return g.rep->done != 0; }

// part[y * n + i] = sum over columns c of chunk y of A(i, c) V(c, j)
__global__ __launch_bounds__(GT) void gm_matvec_partial(GmArgs g, int j) {
  if (stopped(g)) return;
  const int64_t y = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x;
  const int64_t c0 = y * GCHUNK, c1 = min(g.n, c0 + GCHUNK);
  __shared__ double vs[GCHUNK];
  for (int64_t c = c0 + threadIdx.x; c < c1; c += GT) vs[c - c0] = g.V[(int64_t)j * g.n + c];
  __syncthreads();
  if (i >= g.n) return;
  double s0 = 0.0, s1 = 0.0;
  int64_t c = c0;
  for (; c + 1 < c1; c += 2) {
    s0 = fma(g.A[c * g.lda + i], vs[c - c0], s0);
    s1 = fma(g.A[(c + 1) * g.lda + i], vs[c + 1 - c0], s1);
  }
  if (c < c1) s0 = fma(g.A[c * g.lda + i], vs[c - c0], s0);
  g.part[y * g.n + i] = s0 + s1;
}

// z(i) = sum_y part[y * n + i]; rows n..ldz of z (none for square A) untouched
__global__ __launch_bounds__(GT) void gm_matvec_reduce(GmArgs g) {
  if (stopped(g)) return;
  const int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x;
  if (i >= g.n) return;
  const int64_t nch = (g.n + GCHUNK - 1) / GCHUNK;
  double s = 0.0;
  for (int64_t y = 0; y < nch; y++) s += g.part[y * g.n + i];
  g.z[i] = s;
}

// z = M^{-1} r is in g.z: beta = ||z||, V(:,0) = z / beta, g = beta e_1.
__global__ __launch_bounds__(AT) void gm_init(GmArgs g) {
  if (stopped(g)) return;
  __shared__ double red[AT / 64];
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < g.n; i += AT) ss = fma(g.z[i], g.z[i], ss);
  const double beta = sqrt(block_sum_1k(ss, red));
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int64_t i = threadIdx.x; i < g.n; i += AT) g.V[i] = g.z[i] * inv;
  if (threadIdx.x == 0) {
    GmState *s = g.st;
    s->beta = beta;
    s->resid = beta;
    s->j = 0;
    s->inner_done = (beta > 0.0) ? 0 : 1;
    for (int k = 0; k <= g.kmax; k++) g.gv[k] = 0.0;
    g.gv[0] = beta;
  }
}

// Arnoldi step j: z = M^{-1} A v_j is in g.z.  Orthogonalise z against
// v_0..v_j (modified Gram-Schmidt, two sweeps), H(0..j+1, j), v_{j+1}; then
// the Givens rotations reduce H's column j to upper triangular form and
// rotate g.  |g(j+1)| is the preconditioned residual norm of the iterate
// the first j+1 directions give.
__global__ __launch_bounds__(AT) void gm_arnoldi(GmArgs g, int j) {
  if (stopped(g) || g.st->inner_done) return;
  __shared__ double red[AT / 64];
  __shared__ double h[kGmresMax + 1];
  const int64_t n = g.n;
  if (threadIdx.x <= j + 1 && threadIdx.x <= kGmresMax) h[threadIdx.x] = 0.0;
  for (int pass = 0; pass < 2; pass++) {
    __syncthreads();
    // modified Gram-Schmidt sweep; each thread updates its own entries of
    // z, which only it reads in the next dot product
    for (int c = 0; c <= j; c++) {
      double s = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += AT) s = fma(g.V[(int64_t)c * n + i], g.z[i], s);
      const double hc = block_sum_1k(s, red);
      if (threadIdx.x == 0) h[c] += hc;
      for (int64_t i = threadIdx.x; i < n; i += AT) g.z[i] = fma(-hc, g.V[(int64_t)c * n + i], g.z[i]);
    }
  }
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += AT) ss = fma(g.z[i], g.z[i], ss);
  const double hn = sqrt(block_sum_1k(ss, red));
  const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += AT) g.V[(int64_t)(j + 1) * n + i] = g.z[i] * inv;
  __syncthreads();
  if (threadIdx.x == 0) {
    double *H = g.H + (int64_t)j * (g.kmax + 1);  // column j
    for (int c = 0; c <= j; c++) H[c] = h[c];
    H[j + 1] = hn;
    // earlier rotations
    for (int c = 0; c < j; c++) {
      const double a = H[c], b = H[c + 1];
      H[c] = g.cs[c] * a + g.sn[c] * b;
      H[c + 1] = -g.sn[c] * a + g.cs[c] * b;
    }
    // new rotation zeroing H(j+1, j)
    const double a = H[j], b = H[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
    g.cs[j] = c;
    g.sn[j] = s;
    H[j] = r;
    H[j + 1] = 0.0;
    const double gj = g.gv[j];
    g.gv[j] = c * gj;
    g.gv[j + 1] = -s * gj;
    GmState *st = g.st;
    st->j = j + 1;
    st->resid = fabs(g.gv[j + 1]);
    g.rep->krylov_steps += 1;
    if (!(st->resid > g.tol * st->beta) || hn == 0.0 || j + 1 >= g.kmax) st->inner_done = 1;
  }
}

// y = H(0..jn-1, 0..jn-1)^{-1} g(0..jn-1) (upper triangular after the
// rotations), then x += V(:, 0..jn-1) y.
__global__ __launch_bounds__(AT) void gm_update(GmArgs g) {
  if (stopped(g)) return;
  __shared__ double y[kGmresMax];
  const int jn = g.st->j;
  if (threadIdx.x == 0) {
    for (int r = jn - 1; r >= 0; r--) {
      double s = g.gv[r];
      for (int c = r + 1; c < jn; c++) s -= g.H[(int64_t)c * (g.kmax + 1) + r] * y[c];
      const double d = g.H[(int64_t)r * (g.kmax + 1) + r];
      y[r] = (d != 0.0) ? s / d : 0.0;
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < g.n; i += AT) {
    double s = 0.0;
    for (int c = 0; c < jn; c++) s = fma(g.V[(int64_t)c * g.n + i], y[c], s);
    g.x[i] += s;
  }
}

__global__ void gm_count_cycle(GmArgs g) {
  if (threadIdx.x == 0 && !stopped(g)) g.rep->gmres_steps += 1;
}

}  // namespace

size_t gmres_bytes(int64_t n, int kmax) {
  const size_t k1 = (size_t)kmax + 1;
  return 256 + 8 * ((size_t)n * k1 + k1 * kmax + 3 * k1);
}

GmArgs gmres_args(void *mem, int64_t n, int kmax, const double *A, int64_t lda, double *x, double *z,
                  void *partial, RefineState *rep, double tol) {
  GmArgs g{};
  char *p = static_cast<char *>(mem);
  g.st = reinterpret_cast<GmState *>(p);
  double *d = reinterpret_cast<double *>(p + 256);
  const size_t k1 = (size_t)kmax + 1;
  g.V = d;
  g.H = g.V + (size_t)n * k1;
  g.cs = g.H + k1 * kmax;
  g.sn = g.cs + k1;
  g.gv = g.sn + k1;
  g.A = A;
  g.lda = lda;
  g.n = n;
  g.kmax = kmax;
  g.x = x;
  g.z = z;
  g.part = static_cast<double *>(partial);
  g.rep = rep;
  g.tol = tol;
  return g;
}

size_t gmres_partial_bytes(int64_t n) { return (size_t)((n + GCHUNK - 1) / GCHUNK) * n * sizeof(double); }

hipError_t gmres_init(const GmArgs &g, hipStream_t s) {
  hipLaunchKernelGGL(gm_count_cycle, dim3(1), dim3(64), 0, s, g);
  hipLaunchKernelGGL(gm_init, dim3(1), dim3(AT), 0, s, g);
  return hipGetLastError();
}

hipError_t gmres_matvec(const GmArgs &g, int j, hipStream_t s) {
  const int64_t rb = (g.n + GT - 1) / GT, nch = (g.n + GCHUNK - 1) / GCHUNK;
  hipLaunchKernelGGL(gm_matvec_partial, dim3((unsigned)rb, (unsigned)nch), dim3(GT), 0, s, g, j);
  hipLaunchKernelGGL(gm_matvec_reduce, dim3((unsigned)rb), dim3(GT), 0, s, g);
  return hipGetLastError();
}

hipError_t gmres_arnoldi(const GmArgs &g, int j, hipStream_t s) {
  hipLaunchKernelGGL(gm_arnoldi, dim3(1), dim3(AT), 0, s, g, j);
  return hipGetLastError();
}

hipError_t gmres_update(const GmArgs &g, hipStream_t s) {
  hipLaunchKernelGGL(gm_update, dim3(1), dim3(AT), 0, s, g);
  return hipGetLastError();
}

}  // namespace tqr
