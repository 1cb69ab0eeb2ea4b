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
#include "exec_loop.h"

namespace tqr {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;  // threads per workgroup

// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) * B(4x16).  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; register r of lane l holds
// D[4r + l/16][l%16].
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP32-accumulating 16x16 MFMAs (f32 16x16x4 and bf16 16x16x16).  Their
// lane layout differs from the FP64 one: lane l supplies A[l%16][k] and
// B[k][l%16] with k = l/16 (f32) or k = 4(l/16) + e for element e of the
// lane's four bf16 (bf16), and register r of lane l holds
// D[4(l/16) + r][l%16].
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// FP32 -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ s4 to_bf16x4(f4 v) {
  s4 r;
  r[0] = to_bf16(v[0]);
  r[1] = to_bf16(v[1]);
  r[2] = to_bf16(v[2]);
  r[3] = to_bf16(v[3]);
  return r;
}

// Zeroes a loaded value unless `on`, with integer masking.  A select
// between a load and 0 would be turned by the backend into a branch around
// the load followed by a full wait, serialising every load of a loop; the
// mask keeps the (clamped, always in-bounds) load unconditional.
__device__ __forceinline__ double zmask(double v, bool on) {
  return __longlong_as_double(__double_as_longlong(v) & -(long long)on);
}

// threadIdx.x through a volatile register move: values derived from it are
// then recomputed inside each task instead of being hoisted out of the
// persistent loop (where hundreds of them would stay live and spill).
__device__ __forceinline__ int opaque_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

// Reciprocal and square root from the hardware approximations, refined by
// one Newton step each (a few ulps instead of the correctly rounded library
// sequences, which cost several hundred cycles on the panel's serial path).
__device__ __forceinline__ double hrcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double hsqrt(double x) {
  // x > 0 here (a sum of squares with a nonzero term)
  const double y = __builtin_amdgcn_rsq(x);  // ~1/sqrt(x)
  const double h = 0.5 * y;
  double s = x * y;
  const double r = fma(-s, h, 0.5);  // Goldschmidt step
  s = fma(s, r, s);
  const double hh = fma(h, r, h);
  const double d = fma(-s, s, x);
  return fma(d, hh, s);
}

// Sum over aligned groups of G lanes (G = 8 or 16) with DPP lane moves.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(G == 8 || G == 16, "group of 8 or 16 lanes");
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_d<0x141>(v);  // row_half_mirror: lane i <-> 7 - i in each 8
  if (G == 16) v += dpp_d<0x140>(v);  // row_mirror: lane i <-> 15 - i
  return v;
}
template <int G>
__device__ __forceinline__ double group_max(double v) {
  static_assert(G == 8 || G == 16, "group of 8 or 16 lanes");
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  if (G == 16) v = fmax(v, dpp_d<0x140>(v));
  return v;
}

// --------------------------------------------------------------- smem
template <int NB, int IB, int WC>
struct Smem {
  static constexpr int LDV = NB + 2;   // VL column stride
  static constexpr int LDT = IB + 1;   // TL / Ys column stride
  static constexpr int LDW = WC + 16;  // YL row stride
  // reflectors of one block, two buffers: VL[buf][cc*LDV + r].  The solve
  // kernels use VL[1] as YL (a block row of X, YL[kk*LDW + n]).
  static constexpr int VS1 = (IB * LDV > IB * LDW) ? IB * LDV : IB * LDW;
  static constexpr int VS2 = (NB < 64 ? NB : 64) * NB / 2;  // half a column block of R (solve)
  static constexpr int VSZ = VS1 > VS2 ? VS1 : VS2;
  double VL[2][VSZ];
  double TL[2][IB * LDT];              // T of one block: TL[buf][cc*LDT + r] = T(r,cc)
  double vbuf[2][NB + IB];             // panel: current reflector (zero past the panel)
  double Ys[IB * LDT];                 // panel: Ys[jj*LDT + j] = v_jj^T v_j
  double tau[IB];
  int task;
  __device__ double *YL() { return VL[1]; }
};

// The matrices, T factors and right-hand sides are in device memory and
// reached through pointers typed in the global address space.  Plain
// pointers read from the problem table would be generic (flat) to the
// compiler, and flat accesses also count against the LDS wait counter: every
// wait for an LDS operand would then wait for each tile load and store in
// flight as well.
typedef __attribute__((address_space(1))) double gdouble;

enum { M_UNM = 0, M_TT = 1, M_TS = 2 };

// Columns of a chunk handled by one apply pass: 4 waves x 16 columns.
constexpr int CHUNK = 64;

// Loads reflector block b of a tile into VL (rows [rlo, rhi) only), with
// the structure of the mode applied: M_UNM unit lower triangular, M_TT
// upper triangular including the diagonal, M_TS full.  Columns past vcols
// and rows past vrows are zero (no reflector / zero padding).
template <int NB, int IB, int WC, int MODE>
__device__ __forceinline__ void stage_v(const gdouble *__restrict__ V, int64_t ldv, int vrows, int vcols,
                                        int b, int rlo, int rhi, double *VLb) {
  constexpr int TPR = (NT / NB) > 0 ? NT / NB : 1;  // threads per row
  constexpr int CPT = IB / TPR;                      // columns per thread
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  static_assert(CPT * TPR == IB, "IB must split over the threads of a row");
  const int t_ = opaque_tid();
  const int row = t_ % NB;
  const int c0 = (t_ / NB) * CPT;
  if (row >= rlo && row < rhi) {
    const int rowc = min(row, vrows - 1);  // clamped: every load stays inside the tile
#pragma unroll
    for (int u = 0; u < CPT; u++) {
      const int cc = c0 + u, col = b * IB + cc;
      const int colc = min(col, vcols - 1);
      const double ld = V[colc * ldv + rowc];
      const bool in = row < vrows && col < vcols;
      double v;
      if (MODE == M_UNM)
        v = (row == col) ? 1.0 : zmask(ld, row > col && in);
      else if (MODE == M_TT)
        v = zmask(ld, row <= col && in);
      else
        v = zmask(ld, in);
      VLb[cc * LDV + row] = v;
    }
  }
}

// Asynchronous copy of the 128-row segments of reflector block b that meet
// rows [rlo, rhi) straight into LDS (global_load_lds_dwordx4: each lane
// moves two rows, no registers).  Only for full tiles with 16-byte aligned
// columns; the triangular structure is applied when the operands are read.
template <int NB, int IB, int WC>
__device__ __forceinline__ void dma_v(const gdouble *__restrict__ V, int64_t ldv, int b, int rlo, int rhi,
                                      double *VLb) {
  constexpr int SEG = 128;
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  const int wave = __builtin_amdgcn_readfirstlane(opaque_tid() >> 6);
  const int lane = __lane_id();
  const int s0 = rlo / SEG, s1 = (rhi + SEG - 1) / SEG, ns = s1 - s0;
  for (int it = wave; it < IB * ns; it += NT / 64) {
    const int cc = it / ns, seg = s0 + it % ns;
    const gdouble *gp = V + (int64_t)(b * IB + cc) * ldv + seg * SEG + 2 * lane;
    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)gp,
                                     (__attribute__((address_space(3))) void *)(VLb + cc * LDV + seg * SEG),
                                     16, 0, 0);
  }
}

// Structure of reflector block b at (row, reflector column col), applied
// to values read from VL when they were DMA'd raw (staged values are
// already masked).
template <int MODE>
__device__ __forceinline__ double vmask(double v, int row, int col) {
  if (MODE == M_UNM) return row > col ? v : (row == col ? 1.0 : 0.0);
  if (MODE == M_TT) return row <= col ? v : 0.0;
  return v;
}

// ===================================================== block reflector apply
//
// Applies reflector blocks b0..b1-1 of one tile to a chunk of at most CHUNK
// columns:
//   M_UNM: C2 <- Q^T C2 with V unit lower triangular (GEQRT's reflectors)
//   M_TT : [C1; C2] <- Q^T [C1; C2], Q = I - [I; V2] T [I; V2]^T with V2
//          upper triangular (TTQRT's reflectors)
//   M_TS : as M_TT with V2 a full square (TSQRT's reflectors)
// For block b (reflectors b*IB .. b*IB+IB-1):
//   W = V_b^T C2 (+ C1[b rows] for TT/TS),  Y = T_b^T W,
//   C2 -= V_b Y,  C1[b rows] -= Y.
// Each wave owns 16 columns of the chunk and every row of them, so W, Y and
// C2 never leave its registers: C2 and W live in the MFMA accumulator
// layout, whose register s is exactly the B operand of the K-step covering
// rows 4s..4s+3 of a 16-row block.  The reflectors and T are shared through
// LDS.  With `prestaged`, VL/TL already hold block b0 (one block only).
// FB0 >= 0: the blocks are [FB0, FB1), fixed at compile time (b0, b1 are
// ignored), and the block loop is unrolled, so each block's row range, and
// with it which MFMAs run and which operands are loaded, is known to the
// compiler and the loads are scheduled ahead across row blocks.
template <int NB, int IB, int WC, int MODE, int FB0 = -1, int FB1 = -1>
__device__ __forceinline__ void apply_chunk(const gdouble *__restrict__ V, int64_t ldv, int vrows,
                                            int vcols, const gdouble *__restrict__ Tf, gdouble *C1,
                                            int64_t ldc1, gdouble *C2, int64_t ldc2, int c2rows,
                                            int ncols, int b0, int b1, bool prestaged, bool dma,
                                            Smem<NB, IB, WC> &sm) {
  if constexpr (FB0 >= 0) {
    b0 = FB0;
    b1 = FB1;
  }
  constexpr int NRB = NB / 16;
  constexpr int NMB = IB / 16;
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  constexpr int LDT = Smem<NB, IB, WC>::LDT;
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int c = lane & 15;
  const int col = (tid >> 6) * 16 + c;  // this lane's column in the chunk
  const bool ok = col < ncols;

  const int r2lo = (MODE == M_UNM) ? b0 * IB : 0;
  const int r2hi = (MODE == M_TT) ? b1 * IB : NB;
  d4 c2[NRB];
  const int colc = ok ? col : 0;  // clamped: loads of masked lanes stay inside the tile
#pragma unroll
  for (int rb = 0; rb < NRB; rb++) {
    if (rb * 16 + 16 > r2lo && rb * 16 < r2hi) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = rb * 16 + 4 * r + g;
        const double ld = C2[colc * ldc2 + min(row, c2rows - 1)];
        c2[rb][r] = zmask(ld, ok && row >= r2lo && row < r2hi && row < c2rows);
      }
    } else {
      c2[rb] = d4{0.0, 0.0, 0.0, 0.0};
    }
  }

  // T of the next block, loaded into registers while the previous computes
  constexpr int TPT = (IB * IB + NT - 1) / NT;
  double tld[TPT];
  auto load_t = [&](int b) {
#pragma unroll
    for (int q = 0; q < TPT; q++) {
      const int idx = min(tid + NT * q, IB * IB - 1);
      tld[q] = Tf[(b * IB + idx / IB) * IB + idx % IB];
    }
  };
  auto store_t = [&](int buf) {
#pragma unroll
    for (int q = 0; q < TPT; q++) {
      const int idx = tid + NT * q;
      if (idx < IB * IB) {
        const int cc = idx / IB, r = idx % IB;
        sm.TL[buf][cc * LDT + r] = zmask(tld[q], r <= cc);
      }
    }
  };
  auto v_rows = [&](int b, int &rlo, int &rhi) {
    rlo = (MODE == M_UNM) ? b * IB : 0;
    rhi = (MODE == M_TT) ? (b + 1) * IB : NB;
  };
  if (!prestaged) {
    __syncthreads();  // earlier users of VL/TL are done
    int rlo, rhi;
    v_rows(b0, rlo, rhi);
    if (dma) dma_v<NB, IB, WC>(V, ldv, b0, rlo, rhi, sm.VL[0]);
    else stage_v<NB, IB, WC, MODE>(V, ldv, vrows, vcols, b0, rlo, rhi, sm.VL[0]);
    load_t(b0);
  }

  auto block = [&](const int b) {
    const int buf = prestaged ? 0 : ((b - b0) & 1);
    int rlo, rhi;
    v_rows(b, rlo, rhi);
    if (!prestaged) {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this block's DMA / loads landed
      store_t(buf);
      __syncthreads();
      if (b + 1 < b1) {  // prefetch the next block into the other buffer
        int nlo, nhi;
        v_rows(b + 1, nlo, nhi);
        if (dma) dma_v<NB, IB, WC>(V, ldv, b + 1, nlo, nhi, sm.VL[buf ^ 1]);
        else stage_v<NB, IB, WC, MODE>(V, ldv, vrows, vcols, b + 1, nlo, nhi, sm.VL[buf ^ 1]);
        load_t(b + 1);
      }
    }
    const double *VLb = sm.VL[buf];
    const double *TLb = sm.TL[buf];
    const int dlo = b * IB, dhi = (b + 1) * IB;  // rows of the block's triangle
    // W = V_b^T C2, accumulated in two partial sums (even / odd row blocks)
    // so that four independent MFMA chains are in flight
    d4 w[NMB], w2[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) {
      w[mb] = d4{0.0, 0.0, 0.0, 0.0};
      w2[mb] = d4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int rb = 0; rb < NRB; rb++) {
      if (rb * 16 >= rlo && rb * 16 < rhi) {
        const bool diag = dma && MODE != M_TS && rb * 16 >= dlo && rb * 16 < dhi;
#pragma unroll
        for (int s = 0; s < 4; s++) {
#pragma unroll
          for (int mb = 0; mb < NMB; mb++) {
            double a = VLb[(mb * 16 + c) * LDV + rb * 16 + 4 * s + g];
            if (diag) a = vmask<MODE>(a, rb * 16 + 4 * s + g, dlo + mb * 16 + c);
            if (rb & 1)
              w2[mb] = mfma(a, c2[rb][s], w2[mb]);
            else
              w[mb] = mfma(a, c2[rb][s], w[mb]);
          }
        }
      }
    }
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) w[mb] += w2[mb];
    // W += C1[b rows]  (the identity top part of the TT/TS reflectors)
    d4 c1[NMB];
    if (MODE != M_UNM) {
#pragma unroll
      for (int mb = 0; mb < NMB; mb++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = b * IB + mb * 16 + 4 * r + g;
          c1[mb][r] = zmask(C1[colc * ldc1 + row], ok);
        }
        w[mb] += c1[mb];
      }
    }
    // Y = T_b^T W  (T_b upper triangular: block (mb, kb) is zero for kb > mb)
    d4 y[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) {
      y[mb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb <= mb; kb++)
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const double a = TLb[(mb * 16 + c) * LDT + kb * 16 + 4 * s + g];
          y[mb] = mfma(a, w[kb][s], y[mb]);
        }
    }
    if (MODE != M_UNM) {
#pragma unroll
      for (int mb = 0; mb < NMB; mb++) {
        c1[mb] -= y[mb];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = b * IB + mb * 16 + 4 * r + g;
          if (ok) C1[col * ldc1 + row] = c1[mb][r];
        }
      }
    }
    // C2 -= V_b Y
#pragma unroll
    for (int rb = 0; rb < NRB; rb++) {
      if (rb * 16 >= rlo && rb * 16 < rhi) {
        const bool diag = dma && MODE != M_TS && rb * 16 >= dlo && rb * 16 < dhi;
#pragma unroll
        for (int kb = 0; kb < NMB; kb++)
#pragma unroll
          for (int s = 0; s < 4; s++) {
            double a = VLb[(kb * 16 + 4 * s + g) * LDV + rb * 16 + c];
            if (diag) a = vmask<MODE>(a, rb * 16 + c, dlo + kb * 16 + 4 * s + g);
            c2[rb] = mfma(-a, y[kb][s], c2[rb]);
          }
      }
    }
  };
  if constexpr (FB0 >= 0) {
#pragma unroll
    for (int b = FB0; b < FB1; b++) block(b);
  } else {
    for (int b = b0; b < b1; b++) block(b);
  }

#pragma unroll
  for (int rb = 0; rb < NRB; rb++) {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = rb * 16 + 4 * r + g;
      if (ok && row >= r2lo && row < r2hi && row < c2rows) C2[col * ldc2 + row] = c2[rb][r];
    }
  }
}

// ============================================= low-precision reflector apply
//
// apply_chunk's arithmetic with FP32 (P_F32: f32 MFMA) or bfloat16 inputs
// (P_BF16: bf16 MFMA), both accumulating in FP32.  Storage stays FP64: the
// target columns are read from FP64, updated in FP32 registers and written
// back as FP64; V and T are the FP64 values of the panel kernels, rounded
// when they are fed to the MFMA.  Same structure and staging as apply_chunk,
// with the FP32 accumulator layout (lane group g holds rows 4g..4g+3 of a
// 16-row block).
enum { P_F32 = 1, P_BF16 = 2 };

template <int NB, int IB, int WC, int MODE, int P>
__device__ __forceinline__ void apply_chunk_lp(const gdouble *__restrict__ V, int64_t ldv, int vrows,
                                               int vcols, const gdouble *__restrict__ Tf, gdouble *C1,
                                               int64_t ldc1, gdouble *C2, int64_t ldc2, int c2rows,
                                               int ncols, bool dma, Smem<NB, IB, WC> &sm) {
  constexpr int NRB = NB / 16;
  constexpr int NMB = IB / 16;
  const int NBLK = (vcols + IB - 1) / IB;  // blocks that hold reflectors
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  constexpr int LDT = Smem<NB, IB, WC>::LDT;
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int c = lane & 15;
  const int col = (tid >> 6) * 16 + c;
  const bool ok = col < ncols;
  const int colc = ok ? col : 0;

  // the whole apply (every block) touches every row of C2
  f4 c2[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; rb++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = rb * 16 + 4 * g + r;
      c2[rb][r] = (float)zmask(C2[colc * ldc2 + min(row, c2rows - 1)], ok && row < c2rows);
    }

  constexpr int TPT = (IB * IB + NT - 1) / NT;
  double tld[TPT];
  auto load_t = [&](int b) {
#pragma unroll
    for (int q = 0; q < TPT; q++) {
      const int idx = min(tid + NT * q, IB * IB - 1);
      tld[q] = Tf[(b * IB + idx / IB) * IB + idx % IB];
    }
  };
  auto store_t = [&](int buf) {
#pragma unroll
    for (int q = 0; q < TPT; q++) {
      const int idx = tid + NT * q;
      if (idx < IB * IB) {
        const int cc = idx / IB, r = idx % IB;
        sm.TL[buf][cc * LDT + r] = zmask(tld[q], r <= cc);
      }
    }
  };
  auto v_rows = [&](int b, int &rlo, int &rhi) {
    rlo = (MODE == M_UNM) ? b * IB : 0;
    rhi = (MODE == M_TT) ? (b + 1) * IB : NB;
  };
  __syncthreads();
  {
    int rlo, rhi;
    v_rows(0, rlo, rhi);
    if (dma) dma_v<NB, IB, WC>(V, ldv, 0, rlo, rhi, sm.VL[0]);
    else stage_v<NB, IB, WC, MODE>(V, ldv, vrows, vcols, 0, rlo, rhi, sm.VL[0]);
    load_t(0);
  }
  for (int b = 0; b < NBLK; b++) {
    const int buf = b & 1;
    int rlo, rhi;
    v_rows(b, rlo, rhi);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_t(buf);
    __syncthreads();
    if (b + 1 < NBLK) {
      int nlo, nhi;
      v_rows(b + 1, nlo, nhi);
      if (dma) dma_v<NB, IB, WC>(V, ldv, b + 1, nlo, nhi, sm.VL[buf ^ 1]);
      else stage_v<NB, IB, WC, MODE>(V, ldv, vrows, vcols, b + 1, nlo, nhi, sm.VL[buf ^ 1]);
      load_t(b + 1);
    }
    const double *VLb = sm.VL[buf];
    const double *TLb = sm.TL[buf];
    const int dlo = b * IB, dhi = (b + 1) * IB;
    // W = V_b^T C2
    f4 w[NMB], w2[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) {
      w[mb] = f4{0.f, 0.f, 0.f, 0.f};
      w2[mb] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int rb = 0; rb < NRB; rb++) {
      if (rb * 16 >= rlo && rb * 16 < rhi) {
        const bool diag = dma && MODE != M_TS && rb * 16 >= dlo && rb * 16 < dhi;
#pragma unroll
        for (int mb = 0; mb < NMB; mb++) {
          if (P == P_F32) {
#pragma unroll
            for (int s = 0; s < 4; s++) {
              const int row = rb * 16 + 4 * g + s;
              double a = VLb[(mb * 16 + c) * LDV + row];
              if (diag) a = vmask<MODE>(a, row, dlo + mb * 16 + c);
              if (rb & 1) w2[mb] = mfma_f32((float)a, c2[rb][s], w2[mb]);
              else w[mb] = mfma_f32((float)a, c2[rb][s], w[mb]);
            }
          } else {
            s4 av;
#pragma unroll
            for (int e = 0; e < 4; e++) {
              const int row = rb * 16 + 4 * g + e;
              double a = VLb[(mb * 16 + c) * LDV + row];
              if (diag) a = vmask<MODE>(a, row, dlo + mb * 16 + c);
              av[e] = to_bf16((float)a);
            }
            if (rb & 1) w2[mb] = mfma_bf16(av, to_bf16x4(c2[rb]), w2[mb]);
            else w[mb] = mfma_bf16(av, to_bf16x4(c2[rb]), w[mb]);
          }
        }
      }
    }
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) w[mb] += w2[mb];
    f4 c1[NMB];
    if (MODE != M_UNM) {
#pragma unroll
      for (int mb = 0; mb < NMB; mb++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = b * IB + mb * 16 + 4 * g + r;
          c1[mb][r] = (float)zmask(C1[colc * ldc1 + row], ok);
        }
        w[mb] += c1[mb];
      }
    }
    // Y = T_b^T W
    f4 y[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; mb++) {
      y[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb <= mb; kb++) {
        if (P == P_F32) {
#pragma unroll
          for (int s = 0; s < 4; s++) {
            const float a = (float)TLb[(mb * 16 + c) * LDT + kb * 16 + 4 * g + s];
            y[mb] = mfma_f32(a, w[kb][s], y[mb]);
          }
        } else {
          s4 av;
#pragma unroll
          for (int e = 0; e < 4; e++) av[e] = to_bf16((float)TLb[(mb * 16 + c) * LDT + kb * 16 + 4 * g + e]);
          y[mb] = mfma_bf16(av, to_bf16x4(w[kb]), y[mb]);
        }
      }
    }
    if (MODE != M_UNM) {
#pragma unroll
      for (int mb = 0; mb < NMB; mb++) {
        c1[mb] -= y[mb];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int row = b * IB + mb * 16 + 4 * g + r;
          if (ok) C1[col * ldc1 + row] = (double)c1[mb][r];
        }
      }
    }
    // C2 -= V_b Y
#pragma unroll
    for (int rb = 0; rb < NRB; rb++) {
      if (rb * 16 >= rlo && rb * 16 < rhi) {
        const bool diag = dma && MODE != M_TS && rb * 16 >= dlo && rb * 16 < dhi;
#pragma unroll
        for (int kb = 0; kb < NMB; kb++) {
          if (P == P_F32) {
#pragma unroll
            for (int s = 0; s < 4; s++) {
              const int kk = kb * 16 + 4 * g + s;
              double a = VLb[kk * LDV + rb * 16 + c];
              if (diag) a = vmask<MODE>(a, rb * 16 + c, dlo + kk);
              c2[rb] = mfma_f32(-(float)a, y[kb][s], c2[rb]);
            }
          } else {
            s4 av;
#pragma unroll
            for (int e = 0; e < 4; e++) {
              const int kk = kb * 16 + 4 * g + e;
              double a = VLb[kk * LDV + rb * 16 + c];
              if (diag) a = vmask<MODE>(a, rb * 16 + c, dlo + kk);
              av[e] = to_bf16(-(float)a);
            }
            c2[rb] = mfma_bf16(av, to_bf16x4(y[kb]), c2[rb]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int rb = 0; rb < NRB; rb++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = rb * 16 + 4 * g + r;
      if (ok && row < c2rows) C2[col * ldc2 + row] = (double)c2[rb][r];
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
// Panel rows: thread t owns panel column jt = t / RG and rows g, g+RG, ...
// (g = t % RG, RG = 256 / IB contiguous lanes, reduced with DPP).  Panel
// rows are ordered so that the rows whose role changes during the block's
// IB steps come first (the "head"); every later row is a reflector row at
// every step (or zero padding), so the hot loops need no per-row masks:
//   M_UNM: tile rows col0 + pr                       (head: the IB x IB diagonal block)
//   M_TT : [R1 rows col0..col0+IB) [Vt rows col0..col0+IB) [Vt rows 0..col0)
//   M_TS : [R1 rows col0..col0+IB) [Vt rows 0..NB)
// Panel rows of inner block b (the rest of the ordering is zero padding),
// and the row slots per thread that hold them.
template <int NB, int IB, int MODE>
constexpr int panel_rows(int b) {
  return (MODE == M_UNM) ? NB - b * IB : (MODE == M_TT ? 2 * IB + b * IB : IB + NB);
}
template <int NB, int IB, int MODE>
constexpr int panel_slots(int b) {
  constexpr int RG = NT / IB;
  constexpr int PRU = (MODE == M_UNM) ? NB / RG : (NB + IB) / RG;
  const int s = (panel_rows<NB, IB, MODE>(b) + RG - 1) / RG;
  return s < PRU ? s : PRU;
}

// Inner block B of a panel kernel: factor columns [B*IB, (B+1)*IB) (which
// the earlier blocks have updated), write the reflectors and R back, the
// block's T to Tout, and leave V_B in VL[0] and T_B in TL[0] for the
// trailing update.  Compiled per block, each thread carrying only the
// PRU = panel_slots(B) row slots that hold the block's live panel rows
// (TT: 2 IB + B IB rows, GEQRT: NB - B IB), not the whole tile's padding.
template <int NB, int IB, int WC, int MODE, int B>
__device__ __forceinline__ void panel_block(gdouble *Vt, int64_t ldv, int vrows, gdouble *R1,
                                            int64_t ldr, int ncols, gdouble *Tout,
                                            Smem<NB, IB, WC> &sm) {
  constexpr int RG = NT / IB;
  constexpr int PRU = panel_slots<NB, IB, MODE>(B);
  constexpr int UH = ((MODE == M_TT) ? 2 * IB : IB) / RG;  // head slots
  static_assert(PRU >= UH, "every block holds its head rows");
  constexpr int LDV = Smem<NB, IB, WC>::LDV;
  constexpr int LDT = Smem<NB, IB, WC>::LDT;
  const int tid = opaque_tid();
  const int jt = tid / RG;  // panel column of this thread
  const int g = tid % RG;
  {
    constexpr int col0 = B * IB;
    const int col = col0 + jt;
    constexpr int npr = panel_rows<NB, IB, MODE>(B);
    const int colc = min(col, ncols - 1);
    const bool cok = col < ncols;
    // tile row of panel row pr, and which matrix it lives in (true: R1)
    auto prow = [&](int pr, bool &in_r1) {
      in_r1 = (MODE != M_UNM) && pr < IB;
      if (MODE == M_UNM) return col0 + pr;
      if (pr < IB) return col0 + pr;
      if (MODE == M_TT) return pr < 2 * IB ? col0 + pr - IB : pr - 2 * IB;
      return pr - IB;
    };
    double x[PRU];
    // ---- load the panel (clamped addresses, masked with integer AND)
#pragma unroll
    for (int u = 0; u < PRU; u++) {
      const int pr = g + RG * u;
      bool r1;
      const int row = prow(pr, r1);
      if (r1) {
        x[u] = zmask(R1[colc * ldr + row], pr <= jt && cok);
      } else {
        const bool tri = (MODE == M_TT) && pr < 2 * IB;  // R2's diagonal block: upper part only
        x[u] = zmask(Vt[colc * ldv + min(row, vrows - 1)],
                     cok && pr < npr && row < vrows && (!tri || row <= col));
      }
    }
    for (int idx = tid; idx < 2 * RG * PRU; idx += NT) sm.vbuf[idx / (RG * PRU)][idx % (RG * PRU)] = 0.0;
    // role of a head slot at step j: 1 top, 2 reflector row, 0 none
    auto head_role = [&](int pr, int j) -> int {
      if (pr == j) return 1;
      if (MODE == M_UNM) return pr > j ? 2 : 0;
      if (MODE == M_TT) return (pr >= IB && pr - IB <= j) ? 2 : 0;
      return 0;
    };
    // norm of the next reflector column, computed by its own threads one
    // step ahead (fused with their update)
    double sig_n = 0.0, alpha_n = 0.0;
    {
#pragma unroll
      for (int u = 0; u < UH; u++) {
        const int ro = head_role(g + RG * u, 0);
        sig_n += zmask(x[u] * x[u], ro == 2);
        alpha_n += zmask(x[u], ro == 1);
      }
#pragma unroll
      for (int u = UH; u < PRU; u++) sig_n = fma(x[u], x[u], sig_n);
      sig_n = group_sum<RG>(sig_n);
      alpha_n = group_sum<RG>(alpha_n);
    }
    // row jt of the block's T, built during the steps: lane g keeps
    // T(jt, g + RG q) in trow[q]; T(r, j) = tau_j (r = j),
    // -tau_j sum_{r <= c < j} T(r, c) Ys(c, j) (r < j), 0 (r > j), with
    // Ys(c, j) = v_c^T v_j from the dot products of step j.  The groups of
    // the finished columns (jt < j), idle otherwise, form T(jt, j-1) at
    // step j, once the barrier has made Ys(., j-1) complete.
    double trow[IB / RG];
#pragma unroll
    for (int q = 0; q < IB / RG; q++) trow[q] = 0.0;
    auto t_column = [&](int jp) {
      double sp = 0.0;
#pragma unroll
      for (int q = 0; q < IB / RG; q++) {
        const int c = g + RG * q;
        sp += zmask(trow[q] * sm.Ys[c * LDT + jp], c >= jt && c < jp);
      }
      const double ssum = group_sum<RG>(sp);
      const double tj = sm.tau[jp];
      const double v = (jt == jp) ? tj : -tj * ssum;
#pragma unroll
      for (int q = 0; q < IB / RG; q++) trow[q] = (g + RG * q == jp) ? v : trow[q];
    };
    __syncthreads();

    for (int j = 0; j < IB; j++) {
      const int buf = j & 1;
      if (jt == j) {
        const double sig = sig_n, alpha = alpha_n;
        double tau = 0.0, beta = alpha, scale = 0.0;
        const double s2 = fma(alpha, alpha, sig);
        if (sig >= 0x1p-960 && s2 <= 0x1p960) {
          const double nrm = hsqrt(s2);
          beta = (alpha >= 0.0) ? -nrm : nrm;
          tau = (beta - alpha) * hrcp(beta);
          scale = hrcp(alpha - beta);
        } else {
          // The unscaled squares under- or overflow (or the column below
          // the diagonal is zero): ||x|| from the column scaled by a power
          // of two near its largest magnitude.  tau = 0 only when every
          // entry below the diagonal is exactly zero.
          double mx = 0.0;
#pragma unroll
          for (int u = 0; u < UH; u++) mx = fmax(mx, zmask(fabs(x[u]), head_role(g + RG * u, j) == 2));
#pragma unroll
          for (int u = UH; u < PRU; u++) mx = fmax(mx, fabs(x[u]));
          mx = group_max<RG>(mx);
          if (mx > 0.0) {
            int e;
            frexp(fmax(mx, fabs(alpha)), &e);
            double ss = 0.0;
#pragma unroll
            for (int u = 0; u < UH; u++) {
              const double y = ldexp(x[u], -e);
              ss += zmask(y * y, head_role(g + RG * u, j) == 2);
            }
#pragma unroll
            for (int u = UH; u < PRU; u++) {
              const double y = ldexp(x[u], -e);
              ss = fma(y, y, ss);
            }
            ss = group_sum<RG>(ss);
            const double a = ldexp(alpha, -e);
            const double nrm = ldexp(hsqrt(fma(a, a, ss)), e);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) * hrcp(beta);
            scale = hrcp(alpha - beta);
          }
        }
#pragma unroll
        for (int u = 0; u < UH; u++) {
          const int pr = g + RG * u;
          const int ro = head_role(pr, j);
          const double xs = x[u] * scale;
          x[u] = (ro == 2) ? xs : ((ro == 1) ? beta : x[u]);
          sm.vbuf[buf][pr] = (ro == 2) ? xs : ((ro == 1) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = UH; u < PRU; u++) {
          x[u] *= scale;
          sm.vbuf[buf][g + RG * u] = x[u];
        }
        if (g == 0) sm.tau[j] = tau;
      }
      __syncthreads();
      if (jt != j) {
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int u = 0; u < PRU; u += 2) {
          d0 = fma(sm.vbuf[buf][g + RG * u], x[u], d0);
          if (u + 1 < PRU) d1 = fma(sm.vbuf[buf][g + RG * (u + 1)], x[u + 1], d1);
        }
        const double dot = group_sum<RG>(d0 + d1);
        if (jt > j) {
          const double f = sm.tau[j] * dot;
          // update, and the next step's norm for the column it belongs to
          double sg = 0.0, sg2 = 0.0, al = 0.0;
#pragma unroll
          for (int u = 0; u < UH; u++) {
            const int pr = g + RG * u;
            x[u] = fma(-f, sm.vbuf[buf][pr], x[u]);
            const int ro = head_role(pr, j + 1);
            sg += zmask(x[u] * x[u], ro == 2);
            al += zmask(x[u], ro == 1);
          }
#pragma unroll
          for (int u = UH; u < PRU; u++) {
            x[u] = fma(-f, sm.vbuf[buf][g + RG * u], x[u]);
            if (u & 1) sg2 = fma(x[u], x[u], sg2);
            else sg = fma(x[u], x[u], sg);
          }
          if (jt == j + 1) {
            sig_n = group_sum<RG>(sg + sg2);
            alpha_n = group_sum<RG>(al);
          }
        } else {
          if (g == 0) sm.Ys[jt * LDT + j] = dot;  // v_jt^T v_j, jt < j
          if (j > 0) t_column(j - 1);
        }
      }
    }
    __syncthreads();  // Ys(., IB-1) and tau complete
    t_column(IB - 1);


    // ---- write the panel back and stage V_b for the trailing update
#pragma unroll
    for (int u = 0; u < PRU; u++) {
      const int pr = g + RG * u;
      if (pr >= npr) continue;
      bool r1;
      const int row = prow(pr, r1);
      if (MODE == M_UNM) {
        if (row < vrows && cok) Vt[col * ldv + row] = x[u];
        sm.VL[0][jt * LDV + row] = (pr > jt) ? x[u] : (pr == jt ? 1.0 : 0.0);
      } else if (r1) {
        if (pr <= jt && cok) R1[col * ldr + row] = x[u];
      } else {
        const bool mine = (MODE == M_TS) || row <= col;
        if (mine && row < vrows && cok) Vt[col * ldv + row] = x[u];
        sm.VL[0][jt * LDV + row] = mine ? x[u] : 0.0;
      }
    }
    __syncthreads();
    // ---- the block's T (row jt in trow) to LDS for the trailing update
#pragma unroll
    for (int q = 0; q < IB / RG; q++) sm.TL[0][(g + RG * q) * LDT + jt] = trow[q];
    __syncthreads();
    for (int idx = tid; idx < IB * IB; idx += NT) {
      const int cc = idx / IB, r = idx % IB;
      Tout[(col0 + cc) * IB + r] = sm.TL[0][cc * LDT + r];
    }
  }
}

// The trailing update of the tile after inner block B, two levels: block B
// is applied at once (from LDS) only to the rest of its outer block of KOUT
// blocks; when an outer block is complete, its KOUT blocks are applied
// together to every column after it (V and T reloaded, double-buffered), so
// the far columns see few, long MFMA passes instead of one per block.  The
// block ranges are compile-time constants (see apply_chunk).
template <int NB, int IB, int WC, int MODE, int B>
__device__ __forceinline__ void panel_trailing(gdouble *Vt, int64_t ldv, int vrows, gdouble *R1,
                                               int64_t ldr, int ncols, gdouble *Tout,
                                               Smem<NB, IB, WC> &sm) {
  constexpr int NBLK = NB / IB;
  constexpr int KOUT = (128 / IB) < NBLK ? (128 / IB) : NBLK;  // blocks per outer block
  constexpr int col0 = B * IB;
  const int oend = min(ncols, (B / KOUT + 1) * KOUT * IB);
  for (int cs = col0 + IB; cs < oend; cs += CHUNK) {
    const int nc = min(CHUNK, oend - cs);
    apply_chunk<NB, IB, WC, MODE, B, B + 1>(nullptr, 0, vrows, ncols, nullptr,
                                            (MODE == M_UNM) ? nullptr : R1 + cs * ldr, ldr, Vt + cs * ldv,
                                            ldv, vrows, nc, B, B + 1, true, false, sm);
  }
  if constexpr (B % KOUT == KOUT - 1 || B == NBLK - 1) {
    constexpr int F0 = (B / KOUT) * KOUT;
    if (oend < ncols) {
      __syncthreads();  // Vt, R1 and Tout written by every thread
      for (int cs = oend; cs < ncols; cs += CHUNK) {
        const int nc = min(CHUNK, ncols - cs);
        apply_chunk<NB, IB, WC, MODE, F0, B + 1>(Vt, ldv, vrows, ncols, Tout,
                                                 (MODE == M_UNM) ? nullptr : R1 + cs * ldr, ldr,
                                                 Vt + cs * ldv, ldv, vrows, nc, F0, B + 1, false, false, sm);
      }
    }
  }
  __syncthreads();
}

// Runs inner block b (factorization and trailing update) with b fixed at
// compile time.
template <int NB, int IB, int WC, int MODE, int B = 0>
__device__ __forceinline__ void panel_block_at(int b, gdouble *Vt, int64_t ldv, int vrows, gdouble *R1,
                                               int64_t ldr, int ncols, gdouble *Tout,
                                               Smem<NB, IB, WC> &sm) {
  if (b == B) {
    panel_block<NB, IB, WC, MODE, B>(Vt, ldv, vrows, R1, ldr, ncols, Tout, sm);
    panel_trailing<NB, IB, WC, MODE, B>(Vt, ldv, vrows, R1, ldr, ncols, Tout, sm);
    return;
  }
  if constexpr (B + 1 < NB / IB)
    panel_block_at<NB, IB, WC, MODE, B + 1>(b, Vt, ldv, vrows, R1, ldr, ncols, Tout, sm);
}

// Only the inner blocks that hold columns of the matrix are factored (a
// ragged last tile column has ncols < NB); the later blocks hold no
// reflectors and get a zero T.
template <int NB, int IB, int WC, int MODE>
__device__ __forceinline__ void panel_tile(gdouble *Vt, int64_t ldv, int vrows, gdouble *R1,
                                           int64_t ldr, int ncols, gdouble *Tout,
                                           Smem<NB, IB, WC> &sm) {
  const int nblk = (ncols + IB - 1) / IB;
  for (int b = 0; b < nblk; b++) panel_block_at<NB, IB, WC, MODE>(b, Vt, ldv, vrows, R1, ldr, ncols, Tout, sm);
  for (int idx = nblk * IB * IB + opaque_tid(); idx < NB * IB; idx += NT) Tout[idx] = 0.0;
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
__device__ __forceinline__ void gemm_tile(const gdouble *R, int64_t ldr, int nk, const gdouble *X, int64_t ldx,
                          gdouble *C, int64_t ldc, int crows, int ncols, bool trans, Smem<NB, IB, WC> &sm) {
  constexpr int NRB = NB / 16, RBW = (NRB + 3) / 4, NCB = WC / 16;
  constexpr int LDV = Smem<NB, IB, WC>::LDV, LDW = Smem<NB, IB, WC>::LDW;
  const int tid = opaque_tid(), w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
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
    if (!trans) {
      for (int idx = tid; idx < IB * NB; idx += NT) {
        const int cc = idx / NB, r = idx % NB, kc = b * IB + cc;
        sm.VL[0][cc * LDV + r] = (kc < nk) ? R[kc * ldr + r] : 0.0;
      }
    } else {  // R^T: element (r, kc) is R(kc, r); columns r >= crows lie outside the matrix
      for (int idx = tid; idx < IB * NB; idx += NT) {
        const int r = idx / IB, cc = idx % IB, kc = b * IB + cc;
        sm.VL[0][cc * LDV + r] = (kc < nk && r < crows) ? R[r * ldr + kc] : 0.0;
      }
    }
    for (int idx = tid; idx < IB * WC; idx += NT) {
      const int kk = idx / WC, n = idx % WC, kr = b * IB + kk;
      sm.YL()[kk * LDW + n] = (kr < nk && n < ncols) ? X[n * ldx + kr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RBW; t++) {
      const int rb = w + 4 * t;
      if (rb < NRB) {
#pragma unroll
        for (int ks = 0; ks < IB / 4; ks++) {
          const double a = -sm.VL[0][(ks * 4 + g) * LDV + rb * 16 + c];
#pragma unroll
          for (int cb = 0; cb < NCB; cb++)
            acc[t][cb] = mfma(a, sm.YL()[(ks * 4 + g) * LDW + cb * 16 + c], acc[t][cb]);
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
__device__ __forceinline__ void trsm_tile(const gdouble *R, int64_t ldr, int nk, gdouble *X, int64_t ldx, int ncols,
                          int row0, int32_t *singular, Smem<NB, IB, WC> &sm) {
  constexpr int NRB = NB / 16, RBW = (NRB + 3) / 4, NCB = WC / 16, NMB = IB / 16;
  constexpr int LDV = Smem<NB, IB, WC>::LDV, LDT = Smem<NB, IB, WC>::LDT, LDW = Smem<NB, IB, WC>::LDW;
  const int tid = opaque_tid(), w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
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
      sm.TL[0][cc * LDT + r] = (gr < nk && gc < nk && r <= cc) ? R[gc * ldr + gr] : 0.0;
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
              for (int r = 0; r < 4; r++) sm.YL()[(mb * 16 + 4 * r + g) * LDW + cb * 16 + c] = acc[t][cb][r];
    }
    __syncthreads();
    if (tid < WC) {
      const int n = tid;
      for (int r = IB - 1; r >= 0; r--) {
        const int gr = b * IB + r;
        if (gr >= nk) continue;
        double s = sm.YL()[r * LDW + n];
        for (int cc = r + 1; cc < IB && b * IB + cc < nk; cc++) s -= sm.TL[0][cc * LDT + r] * sm.YL()[cc * LDW + n];
        const double d = sm.TL[0][r * LDT + r];
        if (d == 0.0 && n == 0) atomicMin(singular, row0 + gr + 1);
        sm.YL()[r * LDW + n] = s / d;
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
              for (int r = 0; r < 4; r++) acc[t][cb][r] = sm.YL()[(mb * 16 + 4 * r + g) * LDW + cb * 16 + c];
    }
    if (b > 0) {
      // rows above the block: X[0, b*IB) -= R[0, b*IB) x block b
      for (int idx = tid; idx < IB * b * IB; idx += NT) {
        const int cc = idx / (b * IB), r = idx % (b * IB), gc = b * IB + cc;
        sm.VL[0][cc * LDV + r] = (gc < nk) ? R[gc * ldr + r] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < RBW; t++) {
        const int rb = w + 4 * t;
        if (rb < NRB && rb * 16 < b * IB) {
#pragma unroll
          for (int ks = 0; ks < IB / 4; ks++) {
            const double a = -sm.VL[0][(ks * 4 + g) * LDV + rb * 16 + c];
#pragma unroll
            for (int cb = 0; cb < NCB; cb++)
              acc[t][cb] = mfma(a, sm.YL()[(ks * 4 + g) * LDW + cb * 16 + c], acc[t][cb]);
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

// Broadcast of lane l's double (l wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// LDS copy of rows [0, nr) of nc columns of a column-major block:
// dst[cc * NB + row] = src[cc * ld + row].  Each wave takes every fourth
// column, GV_BT columns per batch, and issues the whole batch's loads
// (clamped in bounds, so unconditional) before storing any.
template <int NB>
__device__ __forceinline__ void stage_cols(const gdouble *__restrict__ src, int64_t ld, int nr, int nc,
                                           double *dst) {
  constexpr int U = (NB + 63) / 64;
  constexpr int NW = NT / 64;
  constexpr int BT = 8;
  if (nr <= 0 || nc <= 0) return;
  const int tid = opaque_tid();
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  for (int c0 = w; c0 < nc; c0 += NW * BT) {
    double v[BT][U];
#pragma unroll
    for (int b = 0; b < BT; b++)
#pragma unroll
      for (int u = 0; u < U; u++)
        v[b][u] = src[(int64_t)min(c0 + NW * b, nc - 1) * ld + min(u * 64 + lane, nr - 1)];
#pragma unroll
    for (int b = 0; b < BT; b++)
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int cc = c0 + NW * b, row = u * 64 + lane;
        if (cc < nc && row < nr) dst[cc * NB + row] = v[b][u];
      }
  }
}

// Back-substitution R x = y for a few right-hand sides: one wave per
// column (two at most), each lane holding rows lane, lane + 64, ... in
// registers.  R's columns are staged in LDS 64 at a time (all rows above
// them).  Row r, from the bottom, is finished by its owner lane and
// broadcast with a lane read; every lane then removes its contribution from
// the rows above.  A chain of nk short steps, instead of the blocked
// solve's serial per-column loops; the diagonal's reciprocals are taken
// while a block is staged, so the chain multiplies instead of dividing.
template <int NB, int IB, int WC>
__device__ __forceinline__ void trsm_waves(const gdouble *R, int64_t ldr, int nk, gdouble *X, int64_t ldx,
                                           int ncols, int row0, int32_t *singular, Smem<NB, IB, WC> &sm) {
  constexpr int U = (NB + 63) / 64;  // row groups of 64
  constexpr int CB = NB < 64 ? NB : 64;
  constexpr int CPW = 2;             // columns per wave
  static_assert(2 * Smem<NB, IB, WC>::VSZ >= CB * NB, "LDS too small for a column block of R");
  double *Ls = &sm.VL[0][0];         // VL[0] and VL[1] are contiguous
  double *rinv = &sm.vbuf[0][0];     // reciprocals of the block's diagonal
  static_assert(NB + IB >= CB, "vbuf too small for the diagonal's reciprocals");
  const int tid = opaque_tid();
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  double y[CPW][U];
#pragma unroll
  for (int c = 0; c < CPW; c++) {
    const int n = min(w + (NT / 64) * c, ncols - 1);
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int row = u * 64 + lane;
      y[c][u] = zmask(X[n * ldx + min(row, nk - 1)], row < nk);
    }
  }
#pragma unroll
  for (int ub = U - 1; ub >= 0; ub--) {
    const int c0 = ub * CB;
    if (c0 >= nk) continue;
    const int c1 = min(nk, c0 + CB);
    __syncthreads();  // the previous block's readers are done
    stage_cols<NB>(R + (int64_t)c0 * ldr, ldr, c1, c1 - c0, Ls);
    if (tid < c1 - c0) {  // the block's diagonal: reciprocals, and zero pivots reported
      const double dd = R[(int64_t)(c0 + tid) * ldr + c0 + tid];
      rinv[tid] = 1.0 / dd;
      if (dd == 0.0) atomicMin(singular, row0 + c0 + tid + 1);
    }
    __syncthreads();
    double uc[U], un[U];
    auto load_col = [&](int l, double *dst) {
      const int lc = max(l, 0);
#pragma unroll
      for (int u = 0; u <= ub; u++) dst[u] = Ls[lc * NB + min(u * 64 + lane, c1 - 1)];
    };
    load_col(c1 - 1 - c0, uc);
    double rc = rinv[c1 - 1 - c0];
    for (int l = c1 - 1 - c0; l >= 0; l--) {
      // the next step's column and reciprocal load while this step runs
      load_col(l - 1, un);
      const double rn = rinv[max(l - 1, 0)];
#pragma unroll
      for (int c = 0; c < CPW; c++) {
        const double xr = readlane_d(y[c][ub], l) * rc;
#pragma unroll
        for (int u = 0; u <= ub; u++) {
          if (u < ub)
            y[c][u] = fma(-uc[u], xr, y[c][u]);
          else
            y[c][u] = (lane < l) ? fma(-uc[u], xr, y[c][u]) : ((lane == l) ? xr : y[c][u]);
        }
      }
#pragma unroll
      for (int u = 0; u <= ub; u++) uc[u] = un[u];
      rc = rn;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; c++) {
    const int n = w + (NT / 64) * c;
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int row = u * 64 + lane;
      if (n < ncols && row < nk) X[n * ldx + row] = y[c][u];
    }
  }
}

// Sum over the 64 lanes of a wave, returned (wave-uniform) to every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v = group_sum<16>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// C(r, c) -= sum_kc R(r, kc) X(kc, c)  (trans: R(kc, r)) for at most GV_COLS
// right-hand-side columns: a streaming matrix-vector product (the MFMA tile
// product would spend 16 columns of work on each useful one).  X is staged
// in LDS; R streams from global memory GV_BT columns per wave at a time, all
// loads issued before any is consumed (a single CU needs many bytes in flight
// to approach its share of HBM bandwidth).  Not transposed: wave w takes
// columns kc = w mod 4 with lanes down the rows, and the four waves' partial
// sums meet in LDS.  Transposed: wave w takes columns r = w mod 4 of R with
// lanes down each column, and a wave reduction per right-hand side.
constexpr int GV_COLS = 8;
constexpr int GV_BT = 8;
template <int NB, int IB, int WC>
__device__ __forceinline__ void gemv_tile(const gdouble *R, int64_t ldr, int nk, const gdouble *X, int64_t ldx,
                                          gdouble *C, int64_t ldc, int crows, int ncols, bool trans,
                                          Smem<NB, IB, WC> &sm) {
  constexpr int U = (NB + 63) / 64;
  constexpr int NW = NT / 64;
  static_assert(2 * Smem<NB, IB, WC>::VSZ >= NB * GV_COLS + NW * GV_COLS * NB, "LDS too small for gemv");
  double *xs = &sm.VL[0][0];        // X block, xs[c * NB + kc]
  double *red = xs + NB * GV_COLS;  // partial sums, red[(w * GV_COLS + c) * NB + r]
  const int tid = opaque_tid();
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  if (nk <= 0 || crows <= 0 || ncols <= 0) return;
  __syncthreads();  // earlier users of the LDS are done
  for (int c = 0; c < ncols; c++)
    for (int kc = tid; kc < nk; kc += NT) xs[c * NB + kc] = X[c * ldx + kc];
  __syncthreads();
  double v[GV_BT][U];
  if (!trans) {
    double acc[GV_COLS][U];
#pragma unroll
    for (int c = 0; c < GV_COLS; c++)
#pragma unroll
      for (int u = 0; u < U; u++) acc[c][u] = 0.0;
    for (int k0 = w; k0 < nk; k0 += NW * GV_BT) {
#pragma unroll
      for (int b = 0; b < GV_BT; b++)
#pragma unroll
        for (int u = 0; u < U; u++)
          v[b][u] = R[(int64_t)min(k0 + NW * b, nk - 1) * ldr + min(u * 64 + lane, crows - 1)];
#pragma unroll
      for (int b = 0; b < GV_BT; b++) {
        const int kc = k0 + NW * b;
        if (kc < nk) {
#pragma unroll
          for (int c = 0; c < GV_COLS; c++)
            if (c < ncols) {
              const double xv = xs[c * NB + kc];
#pragma unroll
              for (int u = 0; u < U; u++) acc[c][u] = fma(v[b][u], xv, acc[c][u]);
            }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < GV_COLS; c++)
#pragma unroll
      for (int u = 0; u < U; u++)
        if (c < ncols && u * 64 + lane < NB) red[(w * GV_COLS + c) * NB + u * 64 + lane] = acc[c][u];
    __syncthreads();
    for (int c = 0; c < ncols; c++)
      for (int r = tid; r < crows; r += NT) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NW; q++) sum += red[(q * GV_COLS + c) * NB + r];
        C[c * ldc + r] -= sum;
      }
    return;
  }
  for (int r0 = w; r0 < crows; r0 += NW * GV_BT) {
#pragma unroll
    for (int b = 0; b < GV_BT; b++)
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int kc = u * 64 + lane;
        v[b][u] = zmask(R[(int64_t)min(r0 + NW * b, crows - 1) * ldr + min(kc, nk - 1)], kc < nk);
      }
#pragma unroll
    for (int b = 0; b < GV_BT; b++) {
      const int r = r0 + NW * b;
      if (r < crows) {
#pragma unroll
        for (int c = 0; c < GV_COLS; c++)
          if (c < ncols) {
            double p = 0.0;
#pragma unroll
            for (int u = 0; u < U; u++) p = fma(v[b][u], xs[c * NB + min(u * 64 + lane, nk - 1)], p);
            const double sum = wave_sum(p);
            if (lane == 0) C[c * ldc + r] -= sum;
          }
      }
    }
  }
}

// Forward substitution R^T z = y (R upper triangular, so R^T is lower) for
// right-hand sides in groups of two columns per wave, lanes holding rows as
// in trsm_waves.  Left-looking: row r needs column r of R above the
// diagonal, dotted with the solved part of z (a wave reduction), which keeps
// R's columns contiguous in LDS exactly as the backward solve stages them
// (with the diagonal's reciprocals, as there).
template <int NB, int IB, int WC>
__device__ __forceinline__ void trsmt_waves(const gdouble *R, int64_t ldr, int nk, gdouble *X, int64_t ldx,
                                            int ncols, int row0, int32_t *singular, Smem<NB, IB, WC> &sm) {
  constexpr int U = (NB + 63) / 64;
  constexpr int CB = NB < 64 ? NB : 64;
  constexpr int CPW = 2;
  double *Ls = &sm.VL[0][0];
  double *rinv = &sm.vbuf[0][0];  // reciprocals of the block's diagonal
  const int tid = opaque_tid();
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  for (int cg = 0; cg < ncols; cg += CPW * (NT / 64)) {
    double y[CPW][U], z[CPW][U];
#pragma unroll
    for (int c = 0; c < CPW; c++) {
      const int n = min(cg + w + (NT / 64) * c, ncols - 1);
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int row = u * 64 + lane;
        y[c][u] = zmask(X[n * ldx + min(row, nk - 1)], row < nk);
        z[c][u] = 0.0;
      }
    }
#pragma unroll
    for (int ub = 0; ub < U; ub++) {
      const int c0 = ub * CB;
      if (c0 < nk) {
        const int c1 = min(nk, c0 + CB);
        __syncthreads();
        stage_cols<NB>(R + (int64_t)c0 * ldr, ldr, c1, c1 - c0, Ls);
        if (tid < c1 - c0) {  // the block's diagonal: reciprocals, and zero pivots reported
          const double dd = R[(int64_t)(c0 + tid) * ldr + c0 + tid];
          rinv[tid] = 1.0 / dd;
          if (dd == 0.0) atomicMin(singular, row0 + c0 + tid + 1);
        }
        __syncthreads();
        for (int l = 0; l < c1 - c0; l++) {
          const double *colr = Ls + l * NB;
          double rv[U];
#pragma unroll
          for (int u = 0; u <= ub; u++) rv[u] = colr[min(u * 64 + lane, c1 - 1)];
#pragma unroll
          for (int c = 0; c < CPW; c++) {
            double p = 0.0;
#pragma unroll
            for (int u = 0; u <= ub; u++) p = fma(rv[u], z[c][u], p);  // z is zero from row r on
            const double zr = (readlane_d(y[c][ub], l) - wave_sum(p)) * rinv[l];
            z[c][ub] = (lane == l) ? zr : z[c][ub];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; c++) {
      const int n = cg + w + (NT / 64) * c;
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int row = u * 64 + lane;
        if (n < ncols && row < nk) X[n * ldx + row] = z[c][u];
      }
    }
  }
}

// ================================================================== tasks
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

template <int NB, int IB, int WC>
__device__ __forceinline__ void run_task(const Problem &a, const Task &t, Smem<NB, IB, WC> &sm) {
  if (a.skip && *a.skip) return;
  const int64_t lda = a.lda;
  gdouble *const gA = (gdouble *)a.A;
  gdouble *const gB = (gdouble *)a.B;
  gdouble *const gTf = (gdouble *)a.Tf;
  auto tileA = [&](int i, int j) { return gA + (int64_t)j * NB * lda + (int64_t)i * NB; };
  auto rowsOf = [&](int i) { return (int)min((int64_t)NB, a.m - (int64_t)i * NB); };
  auto Tof = [&](int i, int k, int which) {
    return gTf + (((int64_t)i * a.q + k) * 2 + which) * (int64_t)IB * NB;
  };
  const int kind = t.kind;
  if (kind == K_GEQRT || kind == K_TTQRT || kind == K_TSQRT) {
    const int ncols = (int)min((int64_t)NB, a.n - (int64_t)t.k * NB);
    gdouble *Vt = tileA(t.i, t.k);
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
  if (kind == K_TRSM || kind == K_GEMM || kind == K_TRSMT || kind == K_GEMMT) {
    // right-hand-side tile column j - q; stripe of it
    const int jb = t.j - a.q;
    const int nkk = (int)min((int64_t)NB, a.n - (int64_t)t.k * NB);
    const int ncols = (int)min((int64_t)NB, a.nrhs - (int64_t)jb * NB);
    const int cbeg = t.stripe * a.sw_b;
    const int cend = imin(ncols, cbeg + a.sw_b);
    gdouble *Bc = gB + (int64_t)jb * NB * a.ldb;
    for (int cs = cbeg; cs < cend; cs += WC) {
      const int nc = imin(WC, cend - cs);
      if (kind == K_TRSM && nc <= 2 * (NT / 64))
        trsm_waves<NB, IB, WC>(tileA(t.k, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                               a.ldb, nc, t.k * NB, a.singular, sm);
      else if (kind == K_TRSM)
        trsm_tile<NB, IB, WC>(tileA(t.k, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, nc, t.k * NB, a.singular, sm);
      else if (kind == K_TRSMT)
        trsmt_waves<NB, IB, WC>(tileA(t.k, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                                a.ldb, nc, t.k * NB, a.singular, sm);
      else if (kind == K_GEMM && nc <= GV_COLS)
        gemv_tile<NB, IB, WC>(tileA(t.i, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, Bc + (int64_t)cs * a.ldb + (int64_t)t.i * NB, a.ldb, NB, nc, false, sm);
      else if (kind == K_GEMMT && nc <= GV_COLS)
        gemv_tile<NB, IB, WC>(tileA(t.k, t.i), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, Bc + (int64_t)cs * a.ldb + (int64_t)t.i * NB, a.ldb,
                              (int)min((int64_t)NB, a.n - (int64_t)t.i * NB), nc, true, sm);
      else if (kind == K_GEMM)
        gemm_tile<NB, IB, WC>(tileA(t.i, t.k), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, Bc + (int64_t)cs * a.ldb + (int64_t)t.i * NB, a.ldb, NB, nc, false, sm);
      else  // K_GEMMT: rows of block i (the last one may be ragged) from R(k, i)^T
        gemm_tile<NB, IB, WC>(tileA(t.k, t.i), lda, nkk, Bc + (int64_t)cs * a.ldb + (int64_t)t.k * NB,
                              a.ldb, Bc + (int64_t)cs * a.ldb + (int64_t)t.i * NB, a.ldb,
                              (int)min((int64_t)NB, a.n - (int64_t)t.i * NB), nc, true, sm);
    }
    return;
  }
  // update kinds: target column j (A if j < q, else B)
  gdouble *base;
  int64_t ld;
  int ncols;
  if (t.j < a.q) {
    base = gA + (int64_t)t.j * NB * lda;
    ld = lda;
    ncols = (int)min((int64_t)NB, a.n - (int64_t)t.j * NB);
  } else {
    base = gB + (int64_t)(t.j - a.q) * NB * a.ldb;
    ld = a.ldb;
    ncols = (int)min((int64_t)NB, a.nrhs - (int64_t)(t.j - a.q) * NB);
  }
  const gdouble *V = tileA(t.i, t.k);
  const int vrows = rowsOf(t.i);
  const int vcols = (int)min((int64_t)NB, a.n - (int64_t)t.k * NB);
  const int sw = (t.j < a.q) ? a.sw : a.sw_b;
  const int cbeg = t.stripe * sw;
  const int cend = imin(ncols, cbeg + sw);
  const bool dma = a.dma_ok && NB >= 128 && vrows == NB && vcols == NB;
  const int lp = (t.j < a.q) ? a.update_dtype : 0;  // B's columns always in FP64
  for (int cs = cbeg; cs < cend; cs += CHUNK) {
    const int nc = imin(CHUNK, cend - cs);
    gdouble *C2 = base + (int64_t)cs * ld + (int64_t)t.i * NB;
    if (lp != 0) {
      gdouble *C1 = base + (int64_t)cs * ld + (int64_t)t.piv * NB;
      if (lp == P_F32) {
        if (kind == K_UNMQR)
          apply_chunk_lp<NB, IB, WC, M_UNM, P_F32>(V, lda, vrows, vcols, Tof(t.i, t.k, 0), nullptr, 0, C2, ld,
                                                   vrows, nc, dma, sm);
        else if (kind == K_TTMQR)
          apply_chunk_lp<NB, IB, WC, M_TT, P_F32>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld,
                                                  vrows, nc, dma, sm);
        else
          apply_chunk_lp<NB, IB, WC, M_TS, P_F32>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld,
                                                  vrows, nc, dma, sm);
      } else {
        if (kind == K_UNMQR)
          apply_chunk_lp<NB, IB, WC, M_UNM, P_BF16>(V, lda, vrows, vcols, Tof(t.i, t.k, 0), nullptr, 0, C2,
                                                    ld, vrows, nc, dma, sm);
        else if (kind == K_TTMQR)
          apply_chunk_lp<NB, IB, WC, M_TT, P_BF16>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld,
                                                   vrows, nc, dma, sm);
        else
          apply_chunk_lp<NB, IB, WC, M_TS, P_BF16>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld,
                                                   vrows, nc, dma, sm);
      }
      continue;
    }
    // A ragged last tile column: only its blocks that hold reflectors, with
    // a runtime block loop.
    if (vcols < NB) {
      const int nblk = (vcols + IB - 1) / IB;
      if (kind == K_UNMQR) {
        apply_chunk<NB, IB, WC, M_UNM>(V, lda, vrows, vcols, Tof(t.i, t.k, 0), nullptr, 0, C2, ld, vrows, nc, 0,
                                       nblk, false, dma, sm);
      } else {
        gdouble *C1 = base + (int64_t)cs * ld + (int64_t)t.piv * NB;
        if (kind == K_TTMQR)
          apply_chunk<NB, IB, WC, M_TT>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld, vrows, nc, 0,
                                        nblk, false, dma, sm);
        else
          apply_chunk<NB, IB, WC, M_TS>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld, vrows, nc, 0,
                                        nblk, false, dma, sm);
      }
      continue;
    }
    // Whole-tile applies with the blocks fixed at compile time: one 256 x 64
    // chunk alone on a CU 1.2-1.3x faster than with a runtime block loop.
    if (kind == K_UNMQR) {
      apply_chunk<NB, IB, WC, M_UNM, 0, NB / IB>(V, lda, vrows, vcols, Tof(t.i, t.k, 0), nullptr, 0, C2, ld,
                                             vrows, nc, 0, NB / IB, false, dma, sm);
    } else {
      gdouble *C1 = base + (int64_t)cs * ld + (int64_t)t.piv * NB;
      if (kind == K_TTMQR)
        apply_chunk<NB, IB, WC, M_TT, 0, NB / IB>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld, vrows,
                                              nc, 0, NB / IB, false, dma, sm);
      else
        apply_chunk<NB, IB, WC, M_TS, 0, NB / IB>(V, lda, vrows, vcols, Tof(t.i, t.k, 1), C1, ld, C2, ld, vrows,
                                              nc, 0, NB / IB, false, dma, sm);
    }
  }
}

// ============================================================== executors
// Loads a task descriptor with every field made wave-uniform (scalar), so
// that all loop bounds derived from it are uniform too.
// Resets the executor state (one instance per tile configuration object).
template <int NB>
__global__ void exec_reset(ExecArgs a) {
  executor_reset(a);
}

// Persistent executor over the QR task kinds (the queue protocol is in
// exec_loop.h).
template <int NB, int IB, int WC>
__global__ __launch_bounds__(NT, 1) void exec_persistent(ExecArgs a) {
  __shared__ Smem<NB, IB, WC> sm;
  if (a.skip && *a.skip) return;
  executor_loop(a, &sm.task, [&](const Task &t) __attribute__((always_inline)) {
    run_task<NB, IB, WC>(a.probs ? a.probs[t.prob] : a.prob, t, sm);
  });
}

// Reference executor: one launch runs one task (tasks are launched in a
// topological order on one stream).
template <int NB, int IB, int WC>
__global__ __launch_bounds__(NT, 1) void exec_one(ExecArgs a, int tid) {
  __shared__ Smem<NB, IB, WC> sm;
  if (a.skip && *a.skip) return;
  const int64_t tstart = a.trace ? (int64_t)wall_clock64() : 0;
  {
    const Task t = load_task(a.tasks + tid);
    run_task<NB, IB, WC>(a.probs ? a.probs[t.prob] : a.prob, t, sm);
  }
  __syncthreads();
  if (a.trace && threadIdx.x == 0 && tid < a.trace_cap) {
    int64_t *tr = a.trace + 4 * (int64_t)tid;
    tr[0] = tstart;
    tr[1] = (int64_t)wall_clock64();
    tr[2] = blockIdx.x;
    tr[3] = (int64_t)__smid();
  }
}

template <int NB>
__global__ void exec_finish(ExecArgs a, int32_t *info) {
  if (a.skip && *a.skip) return;
  const int e = a.ctl->error;
  if (a.probs) {  // one info entry per problem
    for (int x = threadIdx.x; x < a.nprob; x += blockDim.x) {
      const int z = *a.probs[x].singular;
      if (info) info[x] = (e != 0) ? e : (z != 0x7fffffff ? z : 0);
    }
    return;
  }
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int z = *a.prob.singular;
    if (info) *info = (e != 0) ? e : (z != 0x7fffffff ? z : 0);
  }
}

// ============================================================ host side
template <int NB, int IB, int WC>
static hipError_t launch_cfg(const ExecArgs &a, int mode, int grid, const int32_t *order,
                             int32_t *info, hipStream_t s) {
  const int rgrid = (int)((a.ntasks + 255) / 256);
  hipLaunchKernelGGL(exec_reset<NB>, dim3(rgrid < 1 ? 1 : (rgrid > 1024 ? 1024 : rgrid)), dim3(256), 0, s, a);
  if (mode == 1) {
    for (int t = 0; t < a.ntasks; t++)
      hipLaunchKernelGGL((exec_one<NB, IB, WC>), dim3(1), dim3(NT), 0, s, a, order[t]);
    hipLaunchKernelGGL(exec_finish<NB>, dim3(1), dim3(64), 0, s, a, info);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((exec_persistent<NB, IB, WC>), dim3(grid), dim3(NT), 0, s, a);
  hipLaunchKernelGGL(exec_finish<NB>, dim3(1), dim3(64), 0, s, a, info);
  return hipGetLastError();
}

template <int NB, int IB, int WC>
static int occupancy_cfg() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, exec_persistent<NB, IB, WC>, NT, 0) != hipSuccess)
    return 1;
  return nb < 1 ? 1 : nb;
}

// This file is compiled once per tile configuration (TQR_CFG_NB,
// TQR_CFG_IB); each object exports that configuration's launch and
// occupancy functions, and configs.cpp dispatches on (nb, ib).
#ifndef TQR_CFG_NB
#error "compile with -DTQR_CFG_NB=<nb> -DTQR_CFG_IB=<ib>"
#endif
#define TQR_FN3(name, a, b) name##_##a##_##b
#define TQR_FN2(name, a, b) TQR_FN3(name, a, b)
#define TQR_FN(name) TQR_FN2(name, TQR_CFG_NB, TQR_CFG_IB)

hipError_t TQR_FN(launch_exec)(const ExecArgs &a, int mode, int grid, const int32_t *order, int32_t *info,
                               hipStream_t s) {
  return launch_cfg<TQR_CFG_NB, TQR_CFG_IB, CHUNK>(a, mode, grid, order, info, s);
}

int TQR_FN(exec_occupancy)() { return occupancy_cfg<TQR_CFG_NB, TQR_CFG_IB, CHUNK>(); }

}  // namespace tqr
