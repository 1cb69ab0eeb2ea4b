// Types shared by the host library and the device executor.
#pragma once
#include <stdint.h>

namespace tqr {

// The six tile kernels of table tab.kernels, plus the two tile kernels of
// the back-substitution R X = C that finishes a least-squares solve.
enum Kind : int32_t {
  K_GEQRT = 0,  // factor square tile (i,k) into R and reflectors V, T
  K_TSQRT = 1,  // zero square tile (i,k) with the triangle of row piv
  K_TTQRT = 2,  // zero triangle (i,k) with the triangle of row piv
  K_UNMQR = 3,  // apply GEQRT(i,k)'s Q^T to tile (i,j)
  K_TSMQR = 4,  // apply TSQRT(i,piv,k)'s Q^T to tiles (piv,j), (i,j)
  K_TTMQR = 5,  // apply TTQRT(i,piv,k)'s Q^T to tiles (piv,j), (i,j)
  K_TRSM = 6,   // X(k,j) <- R(k,k)^{-1} X(k,j)
  K_GEMM = 7,   // X(i,j) <- X(i,j) - R(i,k) X(k,j)
  K_TRSMT = 8,  // X(k,j) <- R(k,k)^{-T} X(k,j)
  K_GEMMT = 9,  // X(i,j) <- X(i,j) - R(k,i)^T X(k,j), i > k
  // tile Cholesky inversion (chapter "Cholesky Inversion", algorithm
  // alg:InPlace), lower triangle in place; W = L^{-1}
  K_POTRF = 10,  // step 1: A(j,j) <- chol(A(j,j))
  K_CTRSM = 11,  //         A(i,j) <- A(i,j) L(j,j)^{-T}
  K_CSYRK = 12,  //         A(j,j) <- A(j,j) - A(j,k) A(j,k)^T
  K_CGEMM = 13,  //         A(i,j) <- A(i,j) - A(i,k) A(j,k)^T
  K_TRTRI = 14,  // step 2: A(j,j) <- L(j,j)^{-1}
  K_TRMML = 15,  //         A(i,j) <- W(i,i) A(i,j)
  K_IGEMM = 16,  //         A(i,j) <- A(i,j) + A(i,k) L(k,j)
  K_TRMMR = 17,  //         A(i,j) <- -A(i,j) W(j,j)
  K_TRMMT = 18,  // step 3: A(i,j) <- W(i,i)^T A(i,j)
  K_LAUUM = 19,  //         A(i,i) <- W(i,i)^T W(i,i)
  K_PGEMM = 20,  //         A(i,j) <- A(i,j) + W(k,i)^T W(k,j)
  K_PSYRK = 21,  //         A(i,i) <- A(i,i) + W(k,i)^T W(k,i)
  K_COUNT = 22
};

// One task of the executor's graph.  Tile coordinates are 0-based; column
// j >= q addresses tile column j - q of the right-hand-side matrix B.  An
// update task covers the column stripe [stripe * sw, (stripe + 1) * sw) of
// its target tiles, sw = nb / stripes.
struct Task {
  int32_t kind;
  int32_t i, piv, k, j;
  int32_t stripe;
  int32_t prob;   // problem index (batched launches), else 0
  int32_t pad1;
};

// Executor control block at the start of the executor-state region.
struct ExecCtl {
  int32_t head;    // next queue slot to pop
  int32_t tail;    // next queue slot to push
  int32_t done;    // tasks finished
  int32_t abort;   // set by the watchdog
  int32_t error;   // 0 or TQR_INFO_TIMEOUT
  int32_t pad[11];  // pad[0]: smallest 1-based index of a zero R(j,j)
};

// One least-squares / factorization problem as the tile kernels see it.
struct Problem {
  double *A;        // the matrix (factored in place)
  int64_t lda, m, n;
  double *B;        // right-hand sides (apply / solve), may be null
  int64_t ldb, nrhs;
  double *Tf;       // T factors: ((i*q + k)*2 + which) * ib * nb doubles
  int32_t p, q;     // tile rows / columns
  int32_t sw;       // stripe width of updates of A's columns (columns per task)
  int32_t sw_b;     // stripe width of tasks on B's columns
  int32_t dma_ok;   // A is 16-byte aligned with even lda: tiles may be DMA'd to LDS
  int32_t update_dtype;  // arithmetic of the updates of A's columns: 0 FP64, 1 FP32, 2 BF16
  int32_t *singular;     // receives min(1-based j) with R(j,j) == 0 (initially 0x7fffffff)
  const int32_t *skip;   // optional: this problem's tasks do nothing while *skip != 0
};

// Everything the device needs for one launch.
struct ExecArgs {
  // graph (library-owned, read-only)
  const Task *tasks;
  const int32_t *succ_off;   // ntasks + 1
  const int32_t *succ;       // successor lists
  const int32_t *indeg0;     // initial dependency counts
  const int32_t *ready0;     // initially ready tasks, priority order
  int32_t ntasks, nready0;
  // nonzero: ready0 lists every task (nready0 == ntasks) in a precomputed
  // order and the queue is filled once by the reset; a finished task only
  // decrements its successors' counts
  int32_t static_order, pad_s;
  // executor state (caller workspace)
  ExecCtl *ctl;
  int32_t *queue;   // ntasks slots
  int32_t *indeg;   // working dependency counts
  // the problem (single launches), or a table indexed by Task::prob (batched)
  Problem prob;
  const Problem *probs;
  int32_t nprob;    // entries of probs
  int32_t pad_;
  int32_t nb, ib;
  int64_t spin_limit;  // watchdog, in wall-clock ticks
  int64_t *trace;      // optional: per task {start, end, workgroup, xcc}
  int64_t trace_cap;   // tasks that fit in `trace`
  const int32_t *skip; // optional: the launch does nothing if *skip != 0
};

}  // namespace tqr
