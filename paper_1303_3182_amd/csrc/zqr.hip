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

constexpr int ZT = 512;  // threads per workgroup: two waves per SIMD

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

// Lane moves and reductions inside a wave without LDS: DPP within each row
// of 16 lanes, readlane across rows (a shuffle would go through LDS, with
// its latency on every step of the chain).
// (every pattern used reads a lane of the same row, always active, so no
// fallback value is needed)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over aligned groups of G lanes (every lane of the wave active): the
// xor-1, xor-2, xor-4 (and xor-8) butterfly, so each lane of a group gets
// the same, order-independent sum.
template <int G>
__device__ __forceinline__ double group_sum_d(double v) {
  static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
  v += dpp_d<0xB1>(v);                // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_d<0x4E>(v);                // quad_perm [2,3,0,1]: lane ^ 2
  if (G >= 8) v += dpp_d<0x141>(v);   // row_half_mirror: the other quad of the 8
  if (G == 16) v += dpp_d<0x140>(v);  // row_mirror: the other half of the row
  return v;
}
// Sum over the 64 lanes of the wave, the same value in every lane.
__device__ __forceinline__ double wave_sum_d(double v) {
  v = group_sum_d<16>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

template <int NB>
struct ZSmem {
  static constexpr int LD = NB + 1;
  static constexpr int CW = NB < 64 ? NB : 64;  // target columns per chunk of the update kernels
  cplx X[NB * LD];               // panel: the tile (GEQRT, zeroed tile); updates: the reflectors
  cplx Y[NB * LD];               // panel: the pivot triangle
  cplx tau[NB];
  double red[ZT / 64];
  int task;
};

// NB x NCOL block of src (rows x cols valid, zero elsewhere) to dst.  Every
// load of the thread is issued before its first LDS store (clamped
// addresses, masked values), so the block costs one memory latency rather
// than one per element.
template <int NB, int NCOL>
__device__ __forceinline__ void zload(const cplx *__restrict__ src, int64_t ld, int rows, int cols, cplx *dst,
                                      int ldd) {
  constexpr int PER = NB * NCOL / ZT;
  static_assert(PER * ZT == NB * NCOL, "a block splits evenly over the threads");
  cplx v[PER];
#pragma unroll
  for (int it = 0; it < PER; it++) {
    const int idx = threadIdx.x + it * ZT;
    const int r = idx % NB, c = idx / NB;
    const bool in = r < rows && c < cols;
    const cplx x = src[(int64_t)(in ? c : 0) * ld + (in ? r : 0)];
    v[it] = in ? x : cplx{0.0, 0.0};
  }
#pragma unroll
  for (int it = 0; it < PER; it++) {
    const int idx = threadIdx.x + it * ZT;
    dst[(idx / NB) * ldd + idx % NB] = v[it];
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
  return {group_sum_d<G>(v.re), group_sum_d<G>(v.im)};
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
      s = wave_sum_d(s);
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
// Applies the nref reflectors of a tile (in LDS, X and tau) to a chunk of
// at most CW target columns (MODE 0: C2 <- H^H C2 with unit lower V; 1 / 2:
// [C1; C2] <- H^H [C1; C2] with V2 upper triangular / full), one reflector
// at a time, with the target chunk in registers: lane g of the
// G lanes of column c holds rows g, g + G, ... of that column of C2 (and of
// C1), loaded from and stored to global memory once per chunk; the
// reflectors stay in LDS (read-only; the G lanes of a row read the same
// address across the wave's columns).
template <int NB, int MODE>
__device__ __forceinline__ void zapply_regs(ZSmem<NB> &sm, cplx *C1g, cplx *C2g, int64_t ld, int vrows, int nref,
                                            int ncc) {
  constexpr int LD = ZSmem<NB>::LD;
  constexpr int CW = ZSmem<NB>::CW;
  constexpr int G = ZT / CW;   // lanes per column
  constexpr int NK = NB / G;   // rows per lane
  const int c = threadIdx.x / G, g = threadIdx.x % G;
  const bool col = c < ncc;
  cplx c2[NK], c1[NK];
#pragma unroll
  for (int k = 0; k < NK; k++) {
    const int q = g + G * k;
    const bool in2 = col && q < vrows;
    const cplx x2 = C2g[(int64_t)(col ? c : 0) * ld + (in2 ? q : 0)];
    c2[k] = in2 ? x2 : cplx{0.0, 0.0};
    if (MODE != 0) {
      const cplx x1 = C1g[(int64_t)(col ? c : 0) * ld + q];
      c1[k] = col ? x1 : cplx{0.0, 0.0};
    }
  }
  // Reflector r = G kr + gr is column r of the staged tile, already zero
  // outside its rows, and rows past vrows of C2 are zero: no per-row guards
  // (exact, the masked terms add zeros).  Its unit entry is row r of C2
  // (MODE 0) or of C1, held by lane gr in slot kr; the slot loop is
  // unrolled, so that slot is a fixed register and only lane gr selects it.
  // this lane's entries of the current reflector; the next one's are
  // loaded while the current one is applied
  cplx xv[NK];
#pragma unroll
  for (int k = 0; k < NK; k++) xv[k] = sm.X[g + G * k];
#pragma unroll
  for (int kr = 0; kr < NK; kr++) {
    if (kr * G < nref) {
      const int gend = min(G, nref - kr * G);
      for (int gr = 0; gr < gend; gr++) {
        const int r = kr * G + gr;
        const int rn = min(r + 1, NB - 1);  // (past the last reflector: loaded, unused)
        cplx xn[NK];
#pragma unroll
        for (int k = 0; k < NK; k++) xn[k] = sm.X[rn * LD + g + G * k];
        cplx w{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < NK; k++) w = cfma_conj(xv[k], c2[k], w);
        const cplx id = (MODE == 0) ? c2[kr] : c1[kr];
        w = cadd(w, (g == gr) ? id : cplx{0.0, 0.0});
        w = group_sum_c<G>(w);
        const cplx f = cmul(conjc(sm.tau[r]), w);
#pragma unroll
        for (int k = 0; k < NK; k++) c2[k] = cfms(f, xv[k], c2[k]);
#pragma unroll
        for (int k = 0; k < NK; k++) xv[k] = xn[k];
        if (MODE == 0)
          c2[kr] = (g == gr) ? csub(c2[kr], f) : c2[kr];
        else
          c1[kr] = (g == gr) ? csub(c1[kr], f) : c1[kr];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NK; k++) {
    const int q = g + G * k;
    if (col && q < vrows) C2g[(int64_t)c * ld + q] = c2[k];
    if (MODE != 0 && col) C1g[(int64_t)c * ld + q] = c1[k];
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
    zload<NB, NB>(tile(t.i, t.k), lda, rows, ncols, sm.X, LD);
    if (kind != K_GEQRT) zload<NB, NB>(tile(t.piv, t.k), lda, NB, ncols, sm.Y, LD);
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
    constexpr int PER = NB * NB / ZT;
    cplx v[PER];
#pragma unroll
    for (int it = 0; it < PER; it++) {  // every load before the first LDS store
      const int idx = threadIdx.x + it * ZT;
      const int r = idx % NB, c = idx / NB;
      const bool in = r < vrows && c < nref && ((mode == 0 && r > c) || (mode == 1 && r <= c) || mode == 2);
      const cplx x = V[(int64_t)(in ? c : 0) * lda + (in ? r : 0)];
      v[it] = in ? x : cplx{0.0, 0.0};
    }
#pragma unroll
    for (int it = 0; it < PER; it++) {
      const int idx = threadIdx.x + it * ZT;
      sm.X[(idx / NB) * LD + idx % NB] = v[it];
    }
    const cplx *tv = tauOf(t.i, t.k, mode == 0 ? 0 : 1);
    for (int x = threadIdx.x; x < NB; x += ZT) sm.tau[x] = (x < nref) ? tv[x] : cplx{0.0, 0.0};
  }
  __syncthreads();  // the reflectors and taus are in LDS
  for (int cs = 0; cs < ncols; cs += CW) {
    const int ncc = min(CW, ncols - cs);
    cplx *C2g = base + (int64_t)cs * ld + (int64_t)t.i * NB;
    cplx *C1g = base + (int64_t)cs * ld + (int64_t)t.piv * NB;
    if (mode == 0)
      zapply_regs<NB, 0>(sm, C1g, C2g, ld, vrows, nref, ncc);
    else if (mode == 1)
      zapply_regs<NB, 1>(sm, C1g, C2g, ld, vrows, nref, ncc);
    else
      zapply_regs<NB, 2>(sm, C1g, C2g, ld, vrows, nref, ncc);
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
