// Tile kernels of the tiled QR factorization (thesis table tab.kernels) and
// the device executor that runs a task graph of them in one persistent
// kernel.  FP64, gfx950.
//
// Data layout: A is column-major with leading dimension lda; tile (i,j)
// starts at A + j*nb*lda + i*nb.  Tiles past m or n are treated as zero
// padded (loads return 0, stores are skipped), which is exact for QR.
// T factors: for tile (i,k), block "which" (0 = GEQRT, 1 = the kernel that
// zeroes the tile) is an ib x nb array, column c holding column c - b*ib of
// the ib x ib upper-triangular T of reflector block b = c / ib.
//
// A workgroup is 256 threads (4 wave64).  Every tile kernel is a device
// function run by one workgroup.
//
// Householder convention (shared with nothing; stated here): for
// x = [alpha; x2], ||x2|| = 0 gives tau = 0; otherwise
// beta = -sign(alpha) ||x|| (sign(0) = +1), tau = (beta - alpha) / beta,
// v = [1; x2 / (alpha - beta)].
#include <hip/hip_runtime.h>

#include "tqr_types.h"

namespace tqr {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;  // threads per workgroup

// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) * B(4x16).  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; register r of lane l holds
// D[4r + l/16][l%16].
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double shfl_xor(double v, int mask) {
  return __shfl_xor(v, mask, 64);
}

// --------------------------------------------------------------- smem
template <int NB, int IB, int WC>
struct Smem {
  static constexpr int LDV = NB + 2;   // VL column stride
  static constexpr int LDT = IB + 1;   // TL / Ys column stride
  static constexpr int LDW = WC + 16;  // WP / YL row stride
  double VL[IB * LDV];                 // reflectors of one block: VL[cc*LDV + r]
  double TL[IB * LDT];                 // T of one block: TL[cc*LDT + r] = T(r,cc)
  double WP[4 * IB * LDW];             // per-wave partial W: WP[(w*IB + kk)*LDW + n]
  double YL[IB * LDW];                 // T^T W: YL[kk*LDW + n]
  double vbuf[2][NB + IB];             // panel: current reflector
  double Ys[IB * LDT];                 // panel: Ys[jj*LDT + j] = v_jj^T v_j
  double tau[IB];
  int task;
};

enum { M_UNM = 0, M_TT = 1, M_TS = 2 };

// ===================================================== block reflector apply
//
// Applies reflector blocks b0..b1-1 of one tile to a chunk of at most WC
// columns:
//   M_UNM: C2 <- Q^T C2 with V unit lower triangular (GEQRT's reflectors)
//   M_TT : [C1; C2] <- Q^T [C1; C2], Q = I - [I; V2] T [I; V2]^T with V2
//          upper triangular (TTQRT's reflectors)
//   M_TS : as M_TT with V2 a full square (TSQRT's reflectors)
// For block b (reflectors b*IB .. b*IB+IB-1):
//   W = V_b^T C2 (+ C1[b rows] for TT/TS),  Y = T_b^T W,
//   C2 -= V_b Y,  C1[b rows] -= Y.
// C1/C2 stay in registers (MFMA accumulator layout) across all blocks; each
// wave owns the 16-row blocks rb = wave + 4t.  With `prestaged`, VL/TL
// already hold block b0 (one block only) and are not reloaded.
template <int NB, int IB, int WC, int MODE>
__device__ void apply_blocks(const double *__restrict__ V, int64_t ldv, int vrows, int vcols,
                             const double *__restrict__ Tf, double *C1, int64_t ldc1,
                             double *C2, int64_t ldc2, int c2rows, int ncols, int b0, int b1,
                             bool prestaged, Smem<NB, IB, WC> &sm) {
  constexpr int NRB = NB / 16;
  constexpr int RBW = (NRB + 3) / 4;
  constexpr int NCB = WC / 16;
  constexpr int NMB = IB / 16;
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  constexpr int LDT = Smem<NB, IB, WC>::LDT;
  constexpr int LDW = Smem<NB, IB, WC>::LDW;
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int c = lane & 15;

  // rows of C2 touched by the blocks
  const int r2lo = (MODE == M_UNM) ? b0 * IB : 0;
  const int r2hi = (MODE == M_TT) ? b1 * IB : NB;
  const int r1lo = b0 * IB, r1hi = b1 * IB;

  d4 c2[RBW][NCB];
  d4 c1[RBW][NCB];
#pragma unroll
  for (int t = 0; t < RBW; t++) {
    const int rb = w + 4 * t;
#pragma unroll
    for (int cb = 0; cb < NCB; cb++) {
      const int col = cb * 16 + c;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = rb * 16 + 4 * r + g;
        double v2 = 0.0, v1 = 0.0;
        if (rb < NRB && col < ncols) {
          if (row >= r2lo && row < r2hi && row < c2rows) v2 = C2[col * ldc2 + row];
          if (MODE != M_UNM && row >= r1lo && row < r1hi) v1 = C1[col * ldc1 + row];
        }
        c2[t][cb][r] = v2;
        c1[t][cb][r] = v1;
      }
    }
  }

  for (int b = b0; b < b1; b++) {
    // rows of V_b that can be nonzero
    const int rlo = (MODE == M_UNM) ? b * IB : 0;
    const int rhi = (MODE == M_TT) ? (b + 1) * IB : NB;
    if (!prestaged) {
      const int nr = rhi - rlo;
      for (int idx = tid; idx < IB * nr; idx += NT) {
        const int cc = idx / nr, r = rlo + idx % nr;
        const int col = b * IB + cc;
        // columns past the matrix hold no reflector (their tau is 0)
        double v = 0.0;
        if (MODE == M_UNM) {
          if (r == col) v = 1.0;
          else if (r > col && r < vrows && col < vcols) v = V[col * ldv + r];
        } else if (MODE == M_TT) {
          if (r <= col && r < vrows && col < vcols) v = V[col * ldv + r];
        } else {
          if (r < vrows && col < vcols) v = V[col * ldv + r];
        }
        sm.VL[cc * LDV + r] = v;
      }
      for (int idx = tid; idx < IB * IB; idx += NT) {
        const int cc = idx / IB, r = idx % IB;
        sm.TL[cc * LDT + r] = (r <= cc) ? Tf[(b * IB + cc) * IB + r] : 0.0;
      }
      __syncthreads();
    }

    // ---- W partial of this wave: V_b[own rows]^T C2[own rows]
    d4 wacc[NMB][NCB];
#pragma unroll
    for (int mb = 0; mb < NMB; mb++)
#pragma unroll
      for (int cb = 0; cb < NCB; cb++) wacc[mb][cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < RBW; t++) {
      const int rb = w + 4 * t;
      if (rb < NRB && rb * 16 >= rlo && rb * 16 < rhi) {
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const int row = rb * 16 + 4 * s + g;  // K index g of K-step s
#pragma unroll
          for (int mb = 0; mb < NMB; mb++) {
            const double a = sm.VL[(mb * 16 + c) * LDV + row];
#pragma unroll
            for (int cb = 0; cb < NCB; cb++) wacc[mb][cb] = mfma(a, c2[t][cb][s], wacc[mb][cb]);
          }
        }
      }
    }
    if (MODE != M_UNM) {
      // W += C1[b*IB .. b*IB+IB) (identity top part of the reflectors)
#pragma unroll
      for (int mb = 0; mb < NMB; mb++) {
        const int rb1 = b * (IB / 16) + mb;
        if ((rb1 & 3) == w) {
          const int t1 = rb1 >> 2;
#pragma unroll
          for (int t = 0; t < RBW; t++)
            if (t == t1)
#pragma unroll
              for (int cb = 0; cb < NCB; cb++) wacc[mb][cb] += c1[t][cb];
        }
      }
    }
#pragma unroll
    for (int mb = 0; mb < NMB; mb++)
#pragma unroll
      for (int cb = 0; cb < NCB; cb++)
#pragma unroll
        for (int r = 0; r < 4; r++)
          sm.WP[(w * IB + mb * 16 + 4 * r + g) * LDW + cb * 16 + c] = wacc[mb][cb][r];
    __syncthreads();

    // ---- W = sum of the partials (in place into WP[0])
    for (int idx = tid; idx < IB * WC; idx += NT) {
      const int kk = idx / WC, n = idx % WC;
      double s = sm.WP[(0 * IB + kk) * LDW + n];
      s += sm.WP[(1 * IB + kk) * LDW + n];
      s += sm.WP[(2 * IB + kk) * LDW + n];
      s += sm.WP[(3 * IB + kk) * LDW + n];
      sm.WP[kk * LDW + n] = s;
    }
    __syncthreads();
    // ---- Y = T_b^T W
    for (int idx = tid; idx < IB * WC; idx += NT) {
      const int i = idx / WC, n = idx % WC;
      double s = 0.0;
      for (int kk = 0; kk <= i; kk++) s += sm.TL[i * LDT + kk] * sm.WP[kk * LDW + n];
      sm.YL[i * LDW + n] = s;
    }
    __syncthreads();

    // ---- C2[own rows] -= V_b[own rows] Y ; C1[b rows] -= Y
#pragma unroll
    for (int t = 0; t < RBW; t++) {
      const int rb = w + 4 * t;
      if (rb < NRB && rb * 16 >= rlo && rb * 16 < rhi) {
#pragma unroll
        for (int ks = 0; ks < IB / 4; ks++) {
          const double a = -sm.VL[(ks * 4 + g) * LDV + rb * 16 + c];
#pragma unroll
          for (int cb = 0; cb < NCB; cb++) {
            const double bb = sm.YL[(ks * 4 + g) * LDW + cb * 16 + c];
            c2[t][cb] = mfma(a, bb, c2[t][cb]);
          }
        }
      }
    }
    if (MODE != M_UNM) {
#pragma unroll
      for (int mb = 0; mb < NMB; mb++) {
        const int rb1 = b * (IB / 16) + mb;
        if ((rb1 & 3) == w) {
          const int t1 = rb1 >> 2;
#pragma unroll
          for (int t = 0; t < RBW; t++)
            if (t == t1)
#pragma unroll
              for (int cb = 0; cb < NCB; cb++)
#pragma unroll
                for (int r = 0; r < 4; r++)
                  c1[t][cb][r] -= sm.YL[(mb * 16 + 4 * r + g) * LDW + cb * 16 + c];
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int t = 0; t < RBW; t++) {
    const int rb = w + 4 * t;
#pragma unroll
    for (int cb = 0; cb < NCB; cb++) {
      const int col = cb * 16 + c;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = rb * 16 + 4 * r + g;
        if (rb < NRB && col < ncols) {
          if (row >= r2lo && row < r2hi && row < c2rows) C2[col * ldc2 + row] = c2[t][cb][r];
          if (MODE != M_UNM && row >= r1lo && row < r1hi) C1[col * ldc1 + row] = c1[t][cb][r];
        }
      }
    }
  }
}

// ============================================================ panel kernels
//
// GEQRT (M_UNM), TTQRT (M_TT), TSQRT (M_TS) on one tile, blocked by IB:
// for each block b the IB panel columns are factored column by column
// (unblocked Householder), the block's T is formed, and the block reflector
// is applied to the tile's remaining columns.
//   M_UNM: Vt is the tile, factored in place into R (upper) and V (lower).
//   M_TT : R1 (pivot row's triangle) on top of Vt's triangle; R1 is
//          overwritten by the new R, Vt's upper triangle by V2 (its lower
//          part, GEQRT's V, is left untouched).
//   M_TS : R1 on top of the full square Vt; Vt becomes V2.
// Panel rows: thread t owns panel column t / RG and rows g, g+RG, ...
// (g = t % RG).  M_UNM panel row pr is tile row b*IB + pr; for TT/TS panel
// rows [0, IB) are R1 rows b*IB + pr and rows [IB, ...) are Vt rows pr - IB.
template <int NB, int IB, int WC, int MODE>
__device__ void panel_tile(double *Vt, int64_t ldv, int vrows, double *R1, int64_t ldr,
                           int ncols, double *Tout, Smem<NB, IB, WC> &sm) {
  constexpr int RG = NT / IB;
  constexpr int PRU = (NB + IB + RG - 1) / RG;
  constexpr int NBLK = NB / IB;
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  constexpr int LDT = Smem<NB, IB, WC>::LDT;
  const int tid = threadIdx.x;
  const int jt = tid / RG;  // panel column of this thread
  const int g = tid % RG;

  for (int b = 0; b < NBLK; b++) {
    const int col0 = b * IB;
    const int col = col0 + jt;
    const int npr = (MODE == M_UNM) ? NB - col0 : (MODE == M_TT ? IB + col0 + IB : IB + NB);
    double x[PRU];
    // ---- load the panel
#pragma unroll
    for (int u = 0; u < PRU; u++) {
      const int pr = g + RG * u;
      double v = 0.0;
      if (pr < npr && col < ncols) {
        if (MODE == M_UNM) {
          const int row = col0 + pr;
          if (row < vrows) v = Vt[col * ldv + row];
        } else if (pr < IB) {
          if (pr <= jt) v = R1[col * ldr + col0 + pr];
        } else {
          const int row = pr - IB;
          if (row < vrows && (MODE == M_TS || row <= col)) v = Vt[col * ldv + row];
        }
      }
      x[u] = v;
    }

    for (int j = 0; j < IB; j++) {
      const int buf = j & 1;
      // role of panel row pr in step j: 1 = top (alpha), 2 = x2, 0 = none
      auto role = [&](int pr) -> int {
        if (pr >= npr) return 0;
        if (MODE == M_UNM) return pr == j ? 1 : (pr > j ? 2 : 0);
        if (pr < IB) return pr == j ? 1 : 0;
        if (MODE == M_TS) return 2;
        return (pr - IB <= col0 + j) ? 2 : 0;
      };
      if (jt == j) {
        double sig = 0.0, alpha = 0.0;
#pragma unroll
        for (int u = 0; u < PRU; u++) {
          const int ro = role(g + RG * u);
          if (ro == 2) sig += x[u] * x[u];
          if (ro == 1) alpha += x[u];
        }
#pragma unroll
        for (int msk = 1; msk < RG; msk <<= 1) {
          sig += shfl_xor(sig, msk);
          alpha += shfl_xor(alpha, msk);
        }
        double tau = 0.0, beta = alpha, scale = 0.0;
        if (sig != 0.0) {
          const double nrm = sqrt(alpha * alpha + sig);
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int u = 0; u < PRU; u++) {
          const int pr = g + RG * u;
          const int ro = role(pr);
          double vv = 0.0;
          if (ro == 2) {
            x[u] *= scale;
            vv = x[u];
          } else if (ro == 1) {
            x[u] = beta;
            vv = 1.0;
          }
          if (pr < npr) sm.vbuf[buf][pr] = vv;
        }
        if (g == 0) sm.tau[j] = tau;
      }
      __syncthreads();
      if (jt != j) {
        double dot = 0.0;
#pragma unroll
        for (int u = 0; u < PRU; u++) {
          const int pr = g + RG * u;
          if (pr < npr) dot += sm.vbuf[buf][pr] * x[u];
        }
#pragma unroll
        for (int msk = 1; msk < RG; msk <<= 1) dot += shfl_xor(dot, msk);
        if (jt > j) {
          const double f = sm.tau[j] * dot;
#pragma unroll
          for (int u = 0; u < PRU; u++) {
            const int pr = g + RG * u;
            if (pr < npr) x[u] -= f * sm.vbuf[buf][pr];
          }
        } else if (g == 0) {
          sm.Ys[jt * LDT + j] = dot;  // v_jt^T v_j, jt < j
        }
      }
    }

    // ---- write the panel back and stage V_b for the trailing update
#pragma unroll
    for (int u = 0; u < PRU; u++) {
      const int pr = g + RG * u;
      if (pr >= npr) continue;
      if (MODE == M_UNM) {
        const int row = col0 + pr;
        if (row < vrows && col < ncols) Vt[col * ldv + row] = x[u];
        sm.VL[jt * LDV + row] = (pr > jt) ? x[u] : (pr == jt ? 1.0 : 0.0);
      } else if (pr < IB) {
        if (pr <= jt && col < ncols) R1[col * ldr + col0 + pr] = x[u];
      } else {
        const int row = pr - IB;
        const bool mine = (MODE == M_TS) || row <= col;
        if (mine && row < vrows && col < ncols) Vt[col * ldv + row] = x[u];
        sm.VL[jt * LDV + row] = mine ? x[u] : 0.0;
      }
    }
    if (MODE == M_UNM) {
      // rows above the block are not part of V_b
      for (int idx = tid; idx < IB * col0; idx += NT) sm.VL[(idx / col0) * LDV + idx % col0] = 0.0;
    } else if (MODE == M_TT) {
      for (int idx = tid; idx < IB * (NB - col0 - IB); idx += NT) {
        const int n2 = NB - col0 - IB;
        sm.VL[(idx / n2) * LDV + col0 + IB + idx % n2] = 0.0;
      }
    }
    __syncthreads();
    // ---- T of the block: T(r,r) = tau_r, T(r,j) = -tau_j sum_c T(r,c) Ys(c,j)
    if (tid < IB) {
      const int r = tid;
      sm.TL[r * LDT + r] = sm.tau[r];
      for (int jj = r + 1; jj < IB; jj++) {
        double s = 0.0;
        for (int cc = r; cc < jj; cc++) s += sm.TL[cc * LDT + r] * sm.Ys[cc * LDT + jj];
        sm.TL[jj * LDT + r] = -sm.tau[jj] * s;
      }
      for (int jj = 0; jj < r; jj++) sm.TL[jj * LDT + r] = 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < IB * IB; idx += NT) {
      const int cc = idx / IB, r = idx % IB;
      Tout[(col0 + cc) * IB + r] = sm.TL[cc * LDT + r];
    }
    // ---- trailing update of the tile's remaining columns with block b
    for (int cs = col0 + IB; cs < NB; cs += WC) {
      const int nc = min(WC, ncols - cs);
      if (nc <= 0) break;
      apply_blocks<NB, IB, WC, MODE>(nullptr, 0, vrows, ncols, nullptr,
                                     (MODE == M_UNM) ? nullptr : R1 + cs * ldr, ldr,
                                     Vt + cs * ldv, ldv, vrows, nc, b, b + 1, true, sm);
    }
    __syncthreads();
  }
}

// ============================================================ solve kernels
//
// Back-substitution tiles for R X = C (C in the right-hand-side matrix):
//   gemm_tile: C(i) -= R(i,k) X(k) for a chunk of <= WC columns;
//   trsm_tile: X(k) = R(k,k)^{-1} C(k), blocked by IB from the bottom, the
//              diagonal IB x IB blocks solved row by row, the rows above
//              updated on MFMA.  Rows >= nk (past n) are left untouched.
// Both keep the chunk in registers in the MFMA accumulator layout.
template <int NB, int IB, int WC>
__device__ void gemm_tile(const double *R, int64_t ldr, int nk, const double *X, int64_t ldx,
                          double *C, int64_t ldc, int crows, int ncols, Smem<NB, IB, WC> &sm) {
  constexpr int NRB = NB / 16, RBW = (NRB + 3) / 4, NCB = WC / 16;
  constexpr int LDV = Smem<NB, IB, WC>::LDV, LDW = Smem<NB, IB, WC>::LDW;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  d4 acc[RBW][NCB];
#pragma unroll
  for (int t = 0; t < RBW; t++)
#pragma unroll
    for (int cb = 0; cb < NCB; cb++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = (w + 4 * t) * 16 + 4 * r + g, col = cb * 16 + c;
        acc[t][cb][r] = (w + 4 * t < NRB && row < crows && col < ncols) ? C[col * ldc + row] : 0.0;
      }
  for (int b = 0; b * IB < nk; b++) {
    for (int idx = tid; idx < IB * NB; idx += NT) {
      const int cc = idx / NB, r = idx % NB, kc = b * IB + cc;
      sm.VL[cc * LDV + r] = (kc < nk) ? R[kc * ldr + r] : 0.0;
    }
    for (int idx = tid; idx < IB * WC; idx += NT) {
      const int kk = idx / WC, n = idx % WC, kr = b * IB + kk;
      sm.YL[kk * LDW + n] = (kr < nk && n < ncols) ? X[n * ldx + kr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RBW; t++) {
      const int rb = w + 4 * t;
      if (rb < NRB) {
#pragma unroll
        for (int ks = 0; ks < IB / 4; ks++) {
          const double a = -sm.VL[(ks * 4 + g) * LDV + rb * 16 + c];
#pragma unroll
          for (int cb = 0; cb < NCB; cb++)
            acc[t][cb] = mfma(a, sm.YL[(ks * 4 + g) * LDW + cb * 16 + c], acc[t][cb]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < RBW; t++)
#pragma unroll
    for (int cb = 0; cb < NCB; cb++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = (w + 4 * t) * 16 + 4 * r + g, col = cb * 16 + c;
        if (w + 4 * t < NRB && row < crows && col < ncols) C[col * ldc + row] = acc[t][cb][r];
      }
}

template <int NB, int IB, int WC>
__device__ void trsm_tile(const double *R, int64_t ldr, int nk, double *X, int64_t ldx, int ncols,
                          int row0, int32_t *singular, Smem<NB, IB, WC> &sm) {
  constexpr int NRB = NB / 16, RBW = (NRB + 3) / 4, NCB = WC / 16, NMB = IB / 16;
  constexpr int LDV = Smem<NB, IB, WC>::LDV, LDT = Smem<NB, IB, WC>::LDT, LDW = Smem<NB, IB, WC>::LDW;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  d4 acc[RBW][NCB];
#pragma unroll
  for (int t = 0; t < RBW; t++)
#pragma unroll
    for (int cb = 0; cb < NCB; cb++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = (w + 4 * t) * 16 + 4 * r + g, col = cb * 16 + c;
        acc[t][cb][r] = (w + 4 * t < NRB && row < nk && col < ncols) ? X[col * ldx + row] : 0.0;
      }
  const int nblk = (nk + IB - 1) / IB;
  for (int b = nblk - 1; b >= 0; b--) {
    // diagonal block of R and the block rows of X into LDS
    for (int idx = tid; idx < IB * IB; idx += NT) {
      const int cc = idx / IB, r = idx % IB;
      const int gr = b * IB + r, gc = b * IB + cc;
      sm.TL[cc * LDT + r] = (gr < nk && gc < nk && r <= cc) ? R[gc * ldr + gr] : 0.0;
    }
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) {
      const int rb = b * (IB / 16) + mb;
      if ((rb & 3) == w)
#pragma unroll
        for (int t = 0; t < RBW; t++)
          if (t == (rb >> 2))
#pragma unroll
            for (int cb = 0; cb < NCB; cb++)
#pragma unroll
              for (int r = 0; r < 4; r++) sm.YL[(mb * 16 + 4 * r + g) * LDW + cb * 16 + c] = acc[t][cb][r];
    }
    __syncthreads();
    if (tid < WC) {
      const int n = tid;
      for (int r = IB - 1; r >= 0; r--) {
        const int gr = b * IB + r;
        if (gr >= nk) continue;
        double s = sm.YL[r * LDW + n];
        for (int cc = r + 1; cc < IB && b * IB + cc < nk; cc++) s -= sm.TL[cc * LDT + r] * sm.YL[cc * LDW + n];
        const double d = sm.TL[r * LDT + r];
        if (d == 0.0 && n == 0) atomicMin(singular, row0 + gr + 1);
        sm.YL[r * LDW + n] = s / d;
      }
    }
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) {
      const int rb = b * (IB / 16) + mb;
      if ((rb & 3) == w)
#pragma unroll
        for (int t = 0; t < RBW; t++)
          if (t == (rb >> 2))
#pragma unroll
            for (int cb = 0; cb < NCB; cb++)
#pragma unroll
              for (int r = 0; r < 4; r++) acc[t][cb][r] = sm.YL[(mb * 16 + 4 * r + g) * LDW + cb * 16 + c];
    }
    if (b > 0) {
      // rows above the block: X[0, b*IB) -= R[0, b*IB) x block b
      for (int idx = tid; idx < IB * b * IB; idx += NT) {
        const int cc = idx / (b * IB), r = idx % (b * IB), gc = b * IB + cc;
        sm.VL[cc * LDV + r] = (gc < nk) ? R[gc * ldr + r] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < RBW; t++) {
        const int rb = w + 4 * t;
        if (rb < NRB && rb * 16 < b * IB) {
#pragma unroll
          for (int ks = 0; ks < IB / 4; ks++) {
            const double a = -sm.VL[(ks * 4 + g) * LDV + rb * 16 + c];
#pragma unroll
            for (int cb = 0; cb < NCB; cb++)
              acc[t][cb] = mfma(a, sm.YL[(ks * 4 + g) * LDW + cb * 16 + c], acc[t][cb]);
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < RBW; t++)
#pragma unroll
    for (int cb = 0; cb < NCB; cb++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = (w + 4 * t) * 16 + 4 * r + g, col = cb * 16 + c;
        if (w + 4 * t < NRB && row < nk && col < ncols) X[col * ldx + row] = acc[t][cb][r];
      }
}

// ================================================================== tasks
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

template <int NB, int IB, int WC>
__device__ void run_task(const ExecArgs &a, const Task &t, Smem<NB, IB, WC> &sm) {
  const int64_t lda = a.lda;
  auto tileA = [&](int i, int j) { return a.A + (int64_t)j * NB * lda + (int64_t)i * NB; };
  auto rowsOf = [&](int i) { return (int)min((int64_t)NB, a.m - (int64_t)i * NB); };
  auto Tof = [&](int i, int k, int which) {
    return a.Tf + (((int64_t)i * a.q + k) * 2 + which) * (int64_t)IB * NB;
  };
  const int kind = t.kind;
  if (kind == K_GEQRT || kind == K_TTQRT || kind == K_TSQRT) {
    const int ncols = (int)min((int64_t)NB, a.n - (int64_t)t.k * NB);
    double *Vt = tileA(t.i, t.k);
    if (kind == K_GEQRT)
      panel_tile<NB, IB, WC, M_UNM>(Vt, lda, rowsOf(t.i), nullptr, 0, ncols, Tof(t.i, t.k, 0), sm);
    else if (kind == K_TTQRT)
      panel_tile<NB, IB, WC, M_TT>(Vt, lda, rowsOf(t.i), tileA(t.piv, t.k), lda, ncols,
                                   Tof(t.i, t.k, 1), sm);
    else
      panel_tile<NB, IB, WC, M_TS>(Vt, lda, rowsOf(t.i), tileA(t.piv, t.k), lda, ncols,
                                   Tof(t.i, t.k, 1), sm);
    return;
  }
  if (kind == K_TRSM || kind == K_GEMM) {
    // right-hand-side tile column j - q; stripe of it
    const int jb = t.j - a.q;
    const int nkk = (int)min((int64_t)NB, a.n - (int64_t)t.k * NB);
    const int ncols = (int)min((int64_t)NB, a.nrhs - (int64_t)jb * NB);
    const int cbeg = t.stripe * a.sw;
    const int cend = imin(ncols, cbeg + a.sw);
    double *Bc = a.B + (int64_t)jb * NB * a.ldb;
    for (int cs = cbeg; cs < cend; cs += WC) {
      const int nc = imin(WC, cend - cs);
      if (kind == K_TRSM)
        trsm_tile<NB, IB, WC>(tileA(t.k, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, nc, t.k * NB, &a.ctl->pad[0], sm);
      else
        gemm_tile<NB, IB, WC>(tileA(t.i, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, Bc + (int64_t)cs * a.ldb + (int64_t)t.i * NB, a.ldb, NB, nc, sm);
    }
    return;
  }
  // update kinds: target column j (A if j < q, else B)
  double *base;
  int64_t ld;
  int ncols;
  if (t.j < a.q) {
    base = a.A + (int64_t)t.j * NB * lda;
    ld = lda;
    ncols = (int)min((int64_t)NB, a.n - (int64_t)t.j * NB);
  } else {
    base = a.B + (int64_t)(t.j - a.q) * NB * a.ldb;
    ld = a.ldb;
    ncols = (int)min((int64_t)NB, a.nrhs - (int64_t)(t.j - a.q) * NB);
  }
  const double *V = tileA(t.i, t.k);
  const int vrows = rowsOf(t.i);
  const int vcols = (int)min((int64_t)NB, a.n - (int64_t)t.k * NB);
  const int cbeg = t.stripe * a.sw;
  const int cend = imin(ncols, cbeg + a.sw);
  for (int cs = cbeg; cs < cend; cs += WC) {
    const int nc = imin(WC, cend - cs);
    double *C2 = base + (int64_t)cs * ld + (int64_t)t.i * NB;
    if (kind == K_UNMQR) {
      apply_blocks<NB, IB, WC, M_UNM>(V, lda, vrows, vcols, Tof(t.i, t.k, 0), nullptr, 0, C2, ld,
                                      vrows, nc, 0, NB / IB, false, sm);
    } else {
      double *C1 = base + (int64_t)cs * ld + (int64_t)t.piv * NB;
      if (kind == K_TTMQR)
        apply_blocks<NB, IB, WC, M_TT>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld, vrows,
                                       nc, 0, NB / IB, false, sm);
      else
        apply_blocks<NB, IB, WC, M_TS>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld, vrows,
                                       nc, 0, NB / IB, false, sm);
    }
  }
}

// ============================================================== executors
// Loads a task descriptor with every field made wave-uniform (scalar), so
// that all loop bounds derived from it are uniform too.
__device__ __forceinline__ Task load_task(const Task *p) {
  Task t = *p;
  t.kind = __builtin_amdgcn_readfirstlane(t.kind);
  t.i = __builtin_amdgcn_readfirstlane(t.i);
  t.piv = __builtin_amdgcn_readfirstlane(t.piv);
  t.k = __builtin_amdgcn_readfirstlane(t.k);
  t.j = __builtin_amdgcn_readfirstlane(t.j);
  t.stripe = __builtin_amdgcn_readfirstlane(t.stripe);
  return t;
}

__device__ __forceinline__ int ld_acquire(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int32_t *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Resets the executor state: dependency counts, queue (initially ready
// tasks first, the rest empty = -1) and control block.
__global__ void exec_reset(ExecArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < a.ntasks; x += stride) {
    a.indeg[x] = a.indeg0[x];
    a.queue[x] = (x < a.nready0) ? a.ready0[x] : -1;
  }
  if (blockIdx.x == 0 && threadIdx.x < 16) {
    int32_t *c = reinterpret_cast<int32_t *>(a.ctl);
    c[threadIdx.x] = 0;
    if (threadIdx.x == 1) c[1] = a.nready0;  // tail
    if (threadIdx.x == 5) c[5] = 0x7fffffff; // smallest 1-based index of a zero R(j,j)
  }
}

// Persistent executor: every workgroup pops queue slots in order, waits for
// the slot to be filled, runs the task, then releases its successors; a
// successor whose count reaches zero is pushed.  Every task is pushed
// exactly once, so a workgroup that pops slot h >= ntasks exits.  A spin
// that exceeds spin_limit sets abort/error and every workgroup exits.
template <int NB, int IB, int WC>
__global__ __launch_bounds__(NT, 1) void exec_persistent(ExecArgs a) {
  __shared__ Smem<NB, IB, WC> sm;
  ExecCtl *ctl = a.ctl;
  for (;;) {
    // Every iteration starts with all threads past their last use of LDS.
    __syncthreads();
    if (threadIdx.x == 0) {
      int task = -1;
      const int h = __hip_atomic_fetch_add(&ctl->head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (h < a.ntasks) {
        const int64_t t0 = wall_clock64();
        for (;;) {
          task = ld_acquire(&a.queue[h]);
          if (task >= 0) break;
          if (ld_relaxed(&ctl->abort)) break;
          if (wall_clock64() - t0 > a.spin_limit) {
            __hip_atomic_store(&ctl->error, -1000, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st_release(&ctl->abort, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      sm.task = task;
    }
    __syncthreads();
    // The task id is wave-uniform; reading it as a scalar makes the loop exit
    // a scalar branch, so no lane can leave the loop while others stay in it.
    const int tid = __builtin_amdgcn_readfirstlane(sm.task);
    if (tid < 0) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    run_task<NB, IB, WC>(a, load_task(a.tasks + tid), sm);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int e = a.succ_off[tid]; e < a.succ_off[tid + 1]; e++) {
        const int s = a.succ[e];
        if (__hip_atomic_fetch_add(&a.indeg[s], -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1) {
          const int slot = __hip_atomic_fetch_add(&ctl->tail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          st_release(&a.queue[slot], s);
        }
      }
      __hip_atomic_fetch_add(&ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Reference executor: one launch runs one task (tasks are launched in a
// topological order on one stream).
template <int NB, int IB, int WC>
__global__ __launch_bounds__(NT, 1) void exec_one(ExecArgs a, int tid) {
  __shared__ Smem<NB, IB, WC> sm;
  run_task<NB, IB, WC>(a, load_task(a.tasks + tid), sm);
}

__global__ void exec_finish(ExecArgs a, int32_t *info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int e = a.ctl->error;
    const int z = a.ctl->pad[0];
    if (info) *info = (e != 0) ? e : (z != 0x7fffffff ? z : 0);
  }
}

// ============================================================ host side
template <int NB, int IB, int WC>
static hipError_t launch_cfg(const ExecArgs &a, int mode, int grid, const int32_t *order,
                             int32_t *info, hipStream_t s) {
  const int rgrid = (int)((a.ntasks + 255) / 256);
  hipLaunchKernelGGL(exec_reset, dim3(rgrid < 1 ? 1 : (rgrid > 1024 ? 1024 : rgrid)), dim3(256), 0, s, a);
  if (mode == 1) {
    for (int t = 0; t < a.ntasks; t++)
      hipLaunchKernelGGL((exec_one<NB, IB, WC>), dim3(1), dim3(NT), 0, s, a, order[t]);
    hipLaunchKernelGGL(exec_finish, dim3(1), dim3(64), 0, s, a, info);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((exec_persistent<NB, IB, WC>), dim3(grid), dim3(NT), 0, s, a);
  hipLaunchKernelGGL(exec_finish, dim3(1), dim3(64), 0, s, a, info);
  return hipGetLastError();
}

template <int NB, int IB, int WC>
static int occupancy_cfg() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, exec_persistent<NB, IB, WC>, NT, 0) != hipSuccess)
    return 1;
  return nb < 1 ? 1 : nb;
}

// Stripe width granule (columns per register-resident chunk) of a config.
int chunk_width(int nb, int ib) {
  (void)ib;
  return nb >= 256 ? 32 : (nb >= 64 ? 64 : 32);
}

#define TQR_CONFIGS(X) \
  X(32, 16, 32)        \
  X(64, 16, 64)        \
  X(64, 32, 64)        \
  X(128, 16, 64)       \
  X(128, 32, 64)       \
  X(256, 16, 32)       \
  X(256, 32, 32)

// mode: 0 persistent, 1 sequential (one launch per task in the host-side
// topological order `order`).
hipError_t launch_exec(const ExecArgs &a, int mode, int grid, const int32_t *order, int32_t *info,
                       hipStream_t s) {
#define X(NB, IB, WC) \
  if (a.nb == NB && a.ib == IB) return launch_cfg<NB, IB, WC>(a, mode, grid, order, info, s);
  TQR_CONFIGS(X)
#undef X
  return hipErrorInvalidValue;
}

int exec_occupancy(int nb, int ib) {
#define X(NB, IB, WC) \
  if (nb == NB && ib == IB) return occupancy_cfg<NB, IB, WC>();
  TQR_CONFIGS(X)
#undef X
  return 0;
}

bool config_supported(int nb, int ib) {
#define X(NB, IB, WC) \
  if (nb == NB && ib == IB) return true;
  TQR_CONFIGS(X)
#undef X
  return false;
}

}  // namespace tqr
