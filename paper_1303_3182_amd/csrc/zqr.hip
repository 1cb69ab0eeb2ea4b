// Double-complex tile kernels of the tiled QR factorization (the thesis's
// "z" workloads, chapter "QR Factorization", section "Experimental
// results") and the persistent executor that runs the same task graph as
// the FP64 path.  gfx950, NB x NB tiles (NB 32 or 64) of a column-major
// complex matrix stored as interleaved (re, im) pairs.
//
// Reflector convention: for x = [alpha; x2], x2 = 0 with alpha real gives
// tau = 0; otherwise beta = -sign(Re alpha) ||x|| (real), tau = (beta -
// alpha) / beta, v = [1; x2 / (alpha - beta)], H = I - tau v v^H and
// H^H x = beta e1.  Q^H acts on a column c as c <- c - conj(tau) v (v^H c),
// reflector 0 first.  tau of the GEQRT of tile (i,k) and of the kernel that
// zeroes it are stored in the workspace, NB complex values each.
//
// Each task stages its tiles (or column chunks of them) in LDS and applies
// the reflectors one at a time: the column's dot products v^H c are summed
// over row slices by groups of lanes and reduced with shuffles.
#include <hip/hip_runtime.h>

#include "exec_loop.h"
#include "tqr_types.h"

namespace tqr {

namespace {

constexpr int ZT = 256;  // threads per workgroup

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx conjc(cplx a) { return {a.re, -a.im}; }
// acc + conj(a) * b
__device__ __forceinline__ cplx cfma_conj(cplx a, cplx b, cplx acc) {
  return {fma(a.re, b.re, fma(a.im, b.im, acc.re)), fma(a.re, b.im, fma(-a.im, b.re, acc.im))};
}
// acc - s * b
__device__ __forceinline__ cplx cfms(cplx s, cplx b, cplx acc) {
  return {fma(-s.re, b.re, fma(s.im, b.im, acc.re)), fma(-s.re, b.im, fma(-s.im, b.re, acc.im))};
}
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm (scaled against overflow)
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ __forceinline__ cplx shfl_xor_c(cplx v, int m) { return {__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64)}; }

template <int NB>
struct ZSmem {
  static constexpr int LD = NB + 1;
  static constexpr int CW = 32;  // target columns per chunk of the update kernels
  static constexpr int YC = (NB > 2 * CW) ? NB : 2 * CW;
  cplx X[NB * LD];               // panel: the tile (GEQRT, zeroed tile); updates: the reflectors
  cplx Y[YC * LD];               // panel: the pivot triangle; updates: target chunks (two of CW columns)
  cplx tau[NB];
  double red[ZT / 64];
  int task;
};

template <int NB>
__device__ __forceinline__ void zload(const cplx *__restrict__ src, int64_t ld, int rows, int cols, cplx *dst,
                                      int ldd, int ncol_alloc) {
  for (int idx = threadIdx.x; idx < NB * ncol_alloc; idx += ZT) {
    const int r = idx % NB, c = idx / NB;
    cplx v{0.0, 0.0};
    if (r < rows && c < cols) v = src[(int64_t)c * ld + r];
    dst[c * ldd + r] = v;
  }
}

template <int NB>
__device__ __forceinline__ void zstore(cplx *__restrict__ dst, int64_t ld, int rows, int cols, const cplx *src,
                                       int lds, int rlo_of_col /* -1: all rows */, bool upper) {
  for (int idx = threadIdx.x; idx < NB * NB; idx += ZT) {
    const int r = idx % NB, c = idx / NB;
    if (r >= rows || c >= cols) continue;
    if (upper && r > c) continue;          // upper triangle only
    if (rlo_of_col >= 0 && r <= c) continue;  // strict lower part only
    dst[(int64_t)c * ld + r] = src[c * lds + r];
  }
}

// Sum of v over the G consecutive lanes of a group (G a power of two <= 64).
template <int G>
__device__ __forceinline__ cplx group_sum_c(cplx v) {
#pragma unroll
  for (int m = 1; m < G; m <<= 1) v = cadd(v, shfl_xor_c(v, m));
  return v;
}

// Reflector of x = [alpha; x2] with ||x2||^2 = s2 (real) and alpha: writes
// tau, beta and the scale 1/(alpha - beta) for v2 = scale * x2.
__device__ __forceinline__ void zlarfg(cplx alpha, double s2, cplx *tau, double *beta, cplx *scale) {
  if (s2 == 0.0 && alpha.im == 0.0) {
    *tau = {0.0, 0.0};
    *beta = alpha.re;
    *scale = {0.0, 0.0};
    return;
  }
  const double nrm = sqrt(fma(alpha.re, alpha.re, fma(alpha.im, alpha.im, s2)));
  const double b = (alpha.re >= 0.0) ? -nrm : nrm;
  *beta = b;
  *tau = {(b - alpha.re) / b, -alpha.im / b};
  *scale = cdiv({1.0, 0.0}, {alpha.re - b, alpha.im});
}

// ---------------------------------------------------------- panel kernels
// Factor the NB columns of the panel held in LDS.  MODE 0 (GEQRT): X is the
// tile (rows x ncols), reflector j lives in rows j..rows-1 of column j.
// MODE 1 (TTQRT) / 2 (TSQRT): Y is the pivot row's upper triangle, X the
// tile zeroed against it (upper triangle for TT, all rows for TS);
// reflector j is [row j of Y; rows 0..j (TT) or 0..rows-1 (TS) of X].
// tau to sm.tau.  One wave computes each reflector; all waves apply it.
template <int NB, int MODE>
__device__ __forceinline__ void zpanel(ZSmem<NB> &sm, int rows, int ncols) {
  constexpr int LD = ZSmem<NB>::LD;
  constexpr int G = ZT / NB;  // lanes per target column in the apply (4 or 8)
  const int lane = threadIdx.x & 63;
  for (int j = 0; j < ncols; j++) {
    // rows of the tile X that the reflector covers
    const int r0 = (MODE == 0) ? j + 1 : 0;
    const int r1 = (MODE == 0) ? rows : (MODE == 1 ? min(j + 1, rows) : rows);
    if (threadIdx.x < 64) {
      double s = 0.0;
      for (int r = r0 + lane; r < r1; r += 64) {
        const cplx x = sm.X[j * LD + r];
        s = fma(x.re, x.re, fma(x.im, x.im, s));
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
      const cplx alpha = (MODE == 0) ? sm.X[j * LD + j] : sm.Y[j * LD + j];
      cplx tau, scale;
      double beta;
      zlarfg(alpha, s, &tau, &beta, &scale);
      for (int r = r0 + lane; r < r1; r += 64) sm.X[j * LD + r] = cmul(sm.X[j * LD + r], scale);
      if (lane == 0) {
        sm.tau[j] = tau;
        if (MODE == 0)
          sm.X[j * LD + j] = {beta, 0.0};
        else
          sm.Y[j * LD + j] = {beta, 0.0};
      }
    }
    __syncthreads();
    // apply H_j^H to columns j+1 .. ncols-1: G lanes per column
    const cplx ctau = conjc(sm.tau[j]);
    for (int c0 = j + 1; c0 < ncols; c0 += ZT / G) {
      const int c = c0 + (int)threadIdx.x / G;
      const int g = threadIdx.x % G;
      cplx w{0.0, 0.0};
      if (c < ncols) {
        for (int r = r0 + g; r < r1; r += G) w = cfma_conj(sm.X[j * LD + r], sm.X[c * LD + r], w);
        if (g == 0) w = cadd(w, (MODE == 0) ? sm.X[c * LD + j] : sm.Y[c * LD + j]);
      }
      w = group_sum_c<G>(w);
      if (c < ncols) {
        const cplx f = cmul(ctau, w);
        for (int r = r0 + g; r < r1; r += G) sm.X[c * LD + r] = cfms(f, sm.X[j * LD + r], sm.X[c * LD + r]);
        if (g == 0) {
          if (MODE == 0)
            sm.X[c * LD + j] = csub(sm.X[c * LD + j], f);
          else
            sm.Y[c * LD + j] = csub(sm.Y[c * LD + j], f);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------- update kernels
// Q^H applied to a chunk of CW target columns held in LDS: MODE 0 (UNMQR):
// C2 only, reflector r = [1 at row r; X rows r+1..vrows-1 of column r];
// MODE 1 (TTMQR) / 2 (TSMQR): [C1; C2], reflector r = [1 at C1's row r;
// X rows 0..r (TT) or 0..vrows-1 (TS) of column r] applied to C2's rows.
template <int NB, int MODE>
__device__ __forceinline__ void zapply_chunk(ZSmem<NB> &sm, cplx *C1, cplx *C2, int vrows, int nref, int ncc) {
  constexpr int LD = ZSmem<NB>::LD;
  constexpr int CW = ZSmem<NB>::CW;
  constexpr int G = ZT / CW;  // 8 lanes per column
  const int c = threadIdx.x / G, g = threadIdx.x % G;
  for (int r = 0; r < nref; r++) {
    const int r0 = (MODE == 0) ? r + 1 : 0;
    const int r1 = (MODE == 0) ? vrows : (MODE == 1 ? min(r + 1, vrows) : vrows);
    cplx w{0.0, 0.0};
    if (c < ncc) {
      for (int q = r0 + g; q < r1; q += G) w = cfma_conj(sm.X[r * LD + q], C2[c * LD + q], w);
      if (g == 0) w = cadd(w, (MODE == 0) ? C2[c * LD + r] : C1[c * LD + r]);
    }
    w = group_sum_c<G>(w);
    if (c < ncc) {
      const cplx f = cmul(conjc(sm.tau[r]), w);
      for (int q = r0 + g; q < r1; q += G) C2[c * LD + q] = cfms(f, sm.X[r * LD + q], C2[c * LD + q]);
      if (g == 0) {
        if (MODE == 0)
          C2[c * LD + r] = csub(C2[c * LD + r], f);
        else
          C1[c * LD + r] = csub(C1[c * LD + r], f);
      }
    }
    __syncthreads();  // (each column's entries belong to one lane group; the
                      // barrier keeps the reflector loop in step for LDS reuse)
  }
}

template <int NB>
__device__ __forceinline__ void run_ztask(const Problem &p, const Task &t, ZSmem<NB> &sm) {
  constexpr int LD = ZSmem<NB>::LD;
  constexpr int CW = ZSmem<NB>::CW;
  cplx *A = reinterpret_cast<cplx *>(p.A);
  cplx *Bm = reinterpret_cast<cplx *>(p.B);
  cplx *taus = reinterpret_cast<cplx *>(p.Tf);
  const int64_t lda = p.lda;
  auto tile = [&](int i, int j) { return A + (int64_t)j * NB * lda + (int64_t)i * NB; };
  auto rowsOf = [&](int i) { return (int)min((int64_t)NB, p.m - (int64_t)i * NB); };
  auto tauOf = [&](int i, int k, int which) { return taus + (((int64_t)i * p.q + k) * 2 + which) * NB; };
  const int kind = t.kind;
  if (kind == K_GEQRT || kind == K_TTQRT || kind == K_TSQRT) {
    const int ncols = (int)min((int64_t)NB, p.n - (int64_t)t.k * NB);
    const int rows = rowsOf(t.i);
    zload<NB>(tile(t.i, t.k), lda, rows, ncols, sm.X, LD, NB);
    if (kind != K_GEQRT) zload<NB>(tile(t.piv, t.k), lda, NB, ncols, sm.Y, LD, NB);
    __syncthreads();
    if (kind == K_GEQRT) {
      zpanel<NB, 0>(sm, rows, ncols);
      zstore<NB>(tile(t.i, t.k), lda, rows, ncols, sm.X, LD, -1, false);
    } else if (kind == K_TTQRT) {
      zpanel<NB, 1>(sm, rows, ncols);
      zstore<NB>(tile(t.piv, t.k), lda, NB, ncols, sm.Y, LD, -1, true);
      zstore<NB>(tile(t.i, t.k), lda, rows, ncols, sm.X, LD, -1, true);  // V2: upper part only
    } else {
      zpanel<NB, 2>(sm, rows, ncols);
      zstore<NB>(tile(t.piv, t.k), lda, NB, ncols, sm.Y, LD, -1, true);
      zstore<NB>(tile(t.i, t.k), lda, rows, ncols, sm.X, LD, -1, false);
    }
    cplx *tau_out = tauOf(t.i, t.k, kind == K_GEQRT ? 0 : 1);
    for (int x = threadIdx.x; x < NB; x += ZT) tau_out[x] = (x < ncols) ? sm.tau[x] : cplx{0.0, 0.0};
    return;
  }
  // updates: target tile column j (A if j < q, else B), reflectors of (i, k)
  cplx *base;
  int64_t ld;
  int ncols;
  if (t.j < p.q) {
    base = A + (int64_t)t.j * NB * lda;
    ld = lda;
    ncols = (int)min((int64_t)NB, p.n - (int64_t)t.j * NB);
  } else {
    base = Bm + (int64_t)(t.j - p.q) * NB * p.ldb;
    ld = p.ldb;
    ncols = (int)min((int64_t)NB, p.nrhs - (int64_t)(t.j - p.q) * NB);
  }
  const int vrows = rowsOf(t.i);
  const int nref = (int)min((int64_t)NB, p.n - (int64_t)t.k * NB);
  const int mode = (kind == K_UNMQR) ? 0 : (kind == K_TTMQR ? 1 : 2);
  // the reflectors, masked to their structure
  {
    const cplx *V = tile(t.i, t.k);
    for (int idx = threadIdx.x; idx < NB * NB; idx += ZT) {
      const int r = idx % NB, c = idx / NB;
      cplx v{0.0, 0.0};
      const bool in = r < vrows && c < nref;
      if (in && ((mode == 0 && r > c) || (mode == 1 && r <= c) || mode == 2)) v = V[(int64_t)c * lda + r];
      sm.X[c * LD + r] = v;
    }
    const cplx *tv = tauOf(t.i, t.k, mode == 0 ? 0 : 1);
    for (int x = threadIdx.x; x < NB; x += ZT) sm.tau[x] = (x < nref) ? tv[x] : cplx{0.0, 0.0};
  }
  cplx *C1s = sm.Y;            // C1 chunk (rows of the pivot tile)
  cplx *C2s = sm.Y + CW * LD;  // C2 chunk
  for (int cs = 0; cs < ncols; cs += CW) {
    const int ncc = min(CW, ncols - cs);
    cplx *C2g = base + (int64_t)cs * ld + (int64_t)t.i * NB;
    cplx *C1g = base + (int64_t)cs * ld + (int64_t)t.piv * NB;
    __syncthreads();
    zload<NB>(C2g, ld, vrows, ncc, C2s, LD, CW);
    if (mode != 0) zload<NB>(C1g, ld, NB, ncc, C1s, LD, CW);
    __syncthreads();
    if (mode == 0)
      zapply_chunk<NB, 0>(sm, C1s, C2s, vrows, nref, ncc);
    else if (mode == 1)
      zapply_chunk<NB, 1>(sm, C1s, C2s, vrows, nref, ncc);
    else
      zapply_chunk<NB, 2>(sm, C1s, C2s, vrows, nref, ncc);
    for (int idx = threadIdx.x; idx < NB * CW; idx += ZT) {
      const int r = idx % NB, c = idx / NB;
      if (c >= ncc) continue;
      if (r < vrows) C2g[(int64_t)c * ld + r] = C2s[c * LD + r];
      if (mode != 0) C1g[(int64_t)c * ld + r] = C1s[c * LD + r];
    }
  }
}

template <int NB>
__global__ void zreset(ExecArgs a) {
  executor_reset(a);
}

template <int NB>
__global__ __launch_bounds__(ZT, 1) void exec_zqr(ExecArgs a) {
  __shared__ ZSmem<NB> sm;
  if (a.skip && *a.skip) return;
  executor_loop(a, &sm.task, [&](const Task &t) __attribute__((always_inline)) { run_ztask<NB>(a.prob, t, sm); });
}

__global__ void zfinish(ExecArgs a, int32_t *info) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && info) *info = a.ctl->error;
}

template <int NB>
hipError_t zlaunch_nb(const ExecArgs &a, int grid, int32_t *info, hipStream_t s) {
  const int rgrid = (int)((a.ntasks + 255) / 256);
  hipLaunchKernelGGL(zreset<NB>, dim3(rgrid < 1 ? 1 : (rgrid > 1024 ? 1024 : rgrid)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(exec_zqr<NB>, dim3(grid), dim3(ZT), 0, s, a);
  hipLaunchKernelGGL(zfinish, dim3(1), dim3(64), 0, s, a, info);
  return hipGetLastError();
}

template <int NB>
int zoccupancy_nb() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, exec_zqr<NB>, ZT, 0) != hipSuccess) return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

bool zqr_nb_supported(int nb) { return nb == 32 || nb == 64; }

int zqr_occupancy(int nb) { return nb == 32 ? zoccupancy_nb<32>() : zoccupancy_nb<64>(); }

hipError_t launch_zqr(const ExecArgs &a, int nb, int grid, int32_t *info, hipStream_t s) {
  if (nb == 32) return zlaunch_nb<32>(a, grid, info, s);
  if (nb == 64) return zlaunch_nb<64>(a, grid, info, s);
  return hipErrorInvalidValue;
}

}  // namespace tqr
