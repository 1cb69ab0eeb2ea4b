/*
 * tqr -- tiled QR factorization on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libtqr.so.  The method is the tiled QR factorization
 * of Bouwmeester's thesis "Tiled Algorithms for Matrix Computations on
 * Multicore Architectures" (2012), chapter "QR Factorization":
 *   - A (m x n, n <= m) = Q R, with R = U_l ... U_1 A built from orthogonal
 *     transformations on tiles (chapter introduction);
 *   - the matrix is viewed as p x q tiles of nb x nb, p = ceil(m/nb),
 *     q = ceil(n/nb) (section "The QR factorization algorithm");
 *   - an elimination list elim(i, piv(i,k), k) fixes which row zeroes which
 *     tile (algorithm alg.QR, section "Elimination lists"); each elimination
 *     runs as the six kernels of table tab.kernels (algorithms alg.elimTR and
 *     alg.elimSQ) and every kernel fires as soon as its inputs are ready
 *     (section "Execution schemes").
 *
 * Conventions shared by every entry point:
 *   - Matrices are FP64, column-major, in device memory, with a leading
 *     dimension (lda >= m).  Every numeric entry point is stream-ordered: it
 *     enqueues work on `stream` and returns without waiting.
 *   - m and n need not be multiples of nb: the last tile row/column is
 *     ragged and is treated as if padded with zeros (exact for QR).
 *   - The caller allocates and owns every buffer.  The library keeps no
 *     pointer to caller memory beyond the enqueued work.  It caches
 *     read-only task tables per shape/options in its own device memory.
 *   - Host-side argument errors return -i for the i-th (1-based) illegal
 *     argument, or one of the TQR_E_* codes below, and enqueue nothing.
 *   - Numerical/executor outcomes are reported asynchronously through an
 *     optional device int32 `info`: 0 ok; j > 0: R(j,j) is exactly zero
 *     (lstsq only; X is then not defined); TQR_INFO_TIMEOUT: the device
 *     watchdog stopped the executor; TQR_INFO_NOCONV: refinement did not
 *     reach its tolerance (X holds the last iterate).
 *   - NaN/Inf in the input propagate; nothing checks for them.
 */
#ifndef TQR_H
#define TQR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Elimination trees (section "Critical paths"): FlatTree = Sameh-Kuck,
 * BinaryTree, Fibonacci = Modi-Clarke order 1, Greedy (algorithm
 * alg.tiled-greedy), GrASAP(i) (definition def.grasap, i = opts.param, 0
 * means 1), PlasmaTree(BS) (BS = opts.param), ASAP on every column.
 * TQR_AUTO lets the learned selector pick tree and nb (falls back to
 * GrASAP with nb = 256). */
enum tqr_tree {
  TQR_FLAT = 0,
  TQR_BINARY = 1,
  TQR_FIBONACCI = 2,
  TQR_GREEDY = 3,
  TQR_GRASAP = 4,
  TQR_PLASMA = 5,
  TQR_ASAP = 6,
  TQR_AUTO = 100
};

/* Kernel families (section "Kernels"): TT triangularises every tile and
 * kills triangles with TTQRT/TTMQR (algorithm alg.elimTR); HYBRID
 * triangularises a row at its first use as a pivot and kills a tile that is
 * still square with TSQRT/TSMQR (algorithm alg.elimSQ), a triangle with
 * TTQRT/TTMQR.  With FlatTree, HYBRID is the pure TS algorithm. */
enum tqr_kernels { TQR_TT = 0, TQR_HYBRID = 1 };

/* Arithmetic of the trailing-update kernels (UNMQR/TSMQR/TTMQR). */
enum tqr_dtype { TQR_F64 = 0, TQR_F32 = 1, TQR_BF16 = 2 };

/* How the task graph is run: one persistent kernel with a device ready
 * queue (default), or one launch per task in list order (reference). */
enum tqr_exec { TQR_EXEC_PERSISTENT = 0, TQR_EXEC_SEQUENTIAL = 1 };

typedef struct tqr_opts {
  int32_t nb;           /* tile size: 32, 64, 128 or 256 (default 256)      */
  int32_t ib;           /* inner block: 16 or 32, divides nb (default 32)   */
  int32_t tree;         /* enum tqr_tree (default TQR_GREEDY)               */
  int32_t kernels;      /* enum tqr_kernels (default TQR_TT)                */
  int32_t param;        /* PlasmaTree BS / GrASAP i (default 0)             */
  int32_t update_dtype; /* enum tqr_dtype (default TQR_F64)                 */
  int32_t exec;         /* enum tqr_exec (default persistent)               */
  int32_t stripes;      /* update tasks per tile (0: 1 up to nb 128, 4 at 256) */
  int32_t max_refine;   /* refinement steps for mixed precision (def. 10)   */
  int32_t priority;     /* enum tqr_priority (default TQR_PRIO_STATIC)      */
  int32_t refine_method;/* enum tqr_refine (default TQR_REFINE_AUTO)        */
  int32_t reserved;     /* 0                                                */
  double refine_tol;    /* refinement stop, relative backward error (0=auto)*/
} tqr_opts;

/* Order in which the executor starts ready tasks (one persistent launch
 * runs a task graph; thesis section "Execution schemes" leaves the order
 * to the runtime):
 *   TQR_PRIO_LIST    one FIFO ready queue, successors in list order;
 *   TQR_PRIO_BOTTOM  one FIFO ready queue, successors and the initially
 *                    ready tasks by decreasing bottom level (longest path
 *                    to the end, tab.kernels weights);
 *   TQR_PRIO_STATIC  (default) the queue filled once, in the start order of
 *                    a critical-path list schedule of the graph simulated
 *                    on the executor's workgroups with estimated GPU task
 *                    durations; workgroups take the tasks in that order,
 *                    each waiting only for its task's predecessors. */
enum tqr_priority { TQR_PRIO_LIST = 0, TQR_PRIO_BOTTOM = 1, TQR_PRIO_STATIC = 2 };

/* Refinement after low-precision updates (tqr_lstsq, one problem):
 * AUTO takes classical steps and, for a square system with one right-hand
 * side, switches to GMRES-based steps once a classical step fails to halve
 * the backward error; CLASSICAL never switches; GMRES uses GMRES-based
 * steps from the first (square, one right-hand side; else classical).  A
 * GMRES-based step that fails to halve the backward error ends the
 * refinement (info: TQR_INFO_NOCONV). */
enum tqr_refine { TQR_REFINE_AUTO = 0, TQR_REFINE_CLASSICAL = 1, TQR_REFINE_GMRES = 2 };

enum {
  TQR_OK = 0,
  TQR_E_HIP = -100,         /* a HIP call failed while enqueueing          */
  TQR_E_WORKSPACE = -101,   /* workspace smaller than tqr_workspace_size   */
  TQR_E_UNSUPPORTED = -102, /* option combination not built                */
  TQR_E_NOMEM = -103,       /* library could not allocate its task tables  */
  TQR_E_INTERNAL = -104,    /* task graph failed its host-side validation  */
  TQR_E_SCRATCH = -105      /* too large for tqr_lstsq_noalloc's scratch   */
};
enum { TQR_INFO_TIMEOUT = -1000, TQR_INFO_NOCONV = -1001 };

/* Fills *o with the defaults listed in tqr_opts. */
void tqr_default_opts(tqr_opts *o);

/* Bytes of device workspace needed by tqr_factor / tqr_factor_ex /
 * tqr_apply_qt (with up to nrhs right-hand sides) for an m x n matrix:
 * the T factors of every factor kernel (two ib x nb blocks per tile, one
 * for GEQRT and one for the kernel that zeroes the tile) plus executor
 * state.  o = NULL means defaults.  Returns 0 for invalid arguments. */
size_t tqr_workspace_size(int64_t m, int64_t n, int64_t nrhs, const tqr_opts *o);

/* Factor A = Q R in place with tile size nb and elimination tree `tree`
 * (other options default; lda = m).  On return (stream-ordered) the upper
 * triangle of the first n rows of A holds R; the other entries and the
 * workspace T hold the Householder vectors and T factors that
 * tqr_apply_qt uses.  T must be tqr_workspace_size(m, n, 0, opts) bytes
 * with opts.nb = nb, opts.tree = tree. */
int tqr_factor(int64_t m, int64_t n, int32_t nb, int32_t tree, double *A, void *T,
               hipStream_t stream);

/* As tqr_factor with explicit lda, workspace size and options.  info: NULL
 * or a device int32 that receives 0 or TQR_INFO_TIMEOUT. */
int tqr_factor_ex(int64_t m, int64_t n, double *A, int64_t lda, void *T, size_t t_bytes,
                  const tqr_opts *o, int32_t *info, hipStream_t stream);

/* B <- Q^T B for the factorization held in (A, T) by a previous factor call
 * with the same m, n and options (the thesis's update kernels UNMQR, TTMQR,
 * TSMQR replayed in list order on the columns of B).  B is m x nrhs,
 * column-major, ldb >= m.  T's factor part is read; its executor part is
 * reused as scratch, so calls on one T must not overlap. */
int tqr_apply_qt(int64_t m, int64_t n, const double *A, int64_t lda, void *T, size_t t_bytes,
                 int64_t nrhs, double *B, int64_t ldb, const tqr_opts *o, int32_t *info,
                 hipStream_t stream);

/* Back-substitution R X = C with the R held in the upper triangle of the
 * first n rows of A by a previous factor call (same m, n, options): C is
 * rows 0..n-1 of B (nrhs columns, ldb >= m), overwritten by X; rows n..m-1
 * of B are not touched.  Least squares needs it after tqr_apply_qt
 * (chapter introduction: x = R^{-1} (Q^T b)(1:n)).  info: NULL or a device
 * int32 receiving 0 or j > 0 if R(j,j) is exactly zero. */
int tqr_solve_r(int64_t m, int64_t n, const double *A, int64_t lda, void *T, size_t t_bytes,
                int64_t nrhs, double *B, int64_t ldb, const tqr_opts *o, int32_t *info,
                hipStream_t stream);

/* Least squares min ||A x - b||_2 for each of nrhs right-hand sides
 * (chapter introduction: QR solves the m-equation, n-unknown least-squares
 * problem): X = R^{-1} (Q^T B)(1:n, :).  A (m x n, lda) and B (m x nrhs,
 * ldb) are not modified; X is n x nrhs (ldx >= n).  Factorization, Q^T B
 * and the back-substitution run as one task graph in one executor launch
 * (B's tile columns are extra columns of the tiled matrix).  work must be
 * tqr_lstsq_work_size bytes.  With opts.update_dtype != TQR_F64 the
 * factorization uses low-precision updates and X is refined in FP64
 * against the caller's A (at most opts.max_refine steps); info then
 * reports TQR_INFO_NOCONV if the tolerance was not reached. */
size_t tqr_lstsq_work_size(int64_t m, int64_t n, int64_t nrhs, const tqr_opts *o);

/* Refinement report, at offset 0 of tqr_lstsq's `work` (device memory,
 * valid once the stream has passed the call).  With update_dtype TQR_F64
 * only `done` = 0 and `iterations` = 0 are written.  Refinement (project
 * addition; the thesis treats FP64 only): square systems take classical
 * iterative refinement, x += R^{-1} (Q^T r)(1:n), or GMRES-based steps
 * (opts.refine_method): the correction solves A d = r by GMRES in FP64
 * left-preconditioned by the computed factors, M^{-1} = R^{-1} Q^T, which
 * converges where kappa(A) times the update precision's unit roundoff
 * exceeds one and classical steps stall; rectangular systems take
 * refinement of the semi-normal equations, x += R^{-1} R^{-T} A^T r.  The
 * residuals r = b - A x and A^T r are FP64 with compensated dot products.
 * Each iteration first tests the backward error of the current x
 * (square: ||r|| / (||A||_F ||x|| + ||b||); rectangular:
 * ||A^T r|| / (||A||_F ||r||)) against opts.refine_tol (0: 16 * 2^-52),
 * worst over the right-hand sides, and stops when it is met.  Unless the
 * stream is being captured into a HIP graph, tqr_lstsq reads the report
 * back after each test (it then returns once the refinement has finished)
 * and enqueues no step after convergence; under capture it enqueues
 * max_refine classical steps, each a no-op once `done` is set. */
#define TQR_REFINE_HISTORY 24
typedef struct tqr_refine_report {
  int32_t done;           /* 1: the tolerance was met                          */
  int32_t iterations;     /* corrections applied before the last test          */
  double backward_error;  /* measured at the last test (-1: none)              */
  double history[TQR_REFINE_HISTORY]; /* at each test (-1: not reached)       */
  int32_t gmres_steps;    /* outer steps taken by GMRES (0: classical only)    */
  int32_t krylov_steps;   /* GMRES iterations (applications of M^{-1} A) in all */
} tqr_refine_report;
int tqr_lstsq(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
              int64_t ldb, double *X, int64_t ldx, void *work, size_t work_bytes,
              const tqr_opts *o, int32_t *info, hipStream_t stream);

/* ---------------------------------------------------- batched least squares
 *
 * Many independent least-squares problems min ||A_x X_x - B_x||, each with
 * its own m_x >= n_x (ragged), nrhs right-hand sides each, in ONE executor
 * launch: the task graphs of all problems form one graph with one ready
 * queue, in the ready order opts.priority selects over the whole graph.
 * Host arrays of sizes and of device pointers; the matrices are device
 * memory, column-major, and are not modified.  Tile size nb/ib come from
 * opts and are shared by the batch; opts.tree = TQR_AUTO picks per problem
 * the tree with the shortest tiled critical path (section "Critical paths")
 * among FlatTree, BinaryTree, Fibonacci, Greedy and GrASAP, else every
 * problem uses opts.tree.  With opts.update_dtype != TQR_F64 each problem
 * is refined in FP64 by the semi-normal equations (see tqr_refine_report);
 * unless the stream is being captured, the reports are read back after
 * each test (the call then synchronises the stream) and no step is
 * enqueued once every problem has converged; the reports of all problems
 * are at the start of `work`, one
 * tqr_refine_report per problem, contiguous.  info: NULL or a device array
 * of count int32 (meaning as for tqr_lstsq).  Arguments: -1 count < 1,
 * -2 bad m / n, -4 nrhs < 1, -5 bad A / lda, -7 bad B / ldb, -9 bad X / ldx,
 * -11 work NULL. */
size_t tqr_lstsq_batched_work_size(int32_t count, const int64_t *m, const int64_t *n, int64_t nrhs,
                                   const tqr_opts *o); /* o->nb == 0: largest over the built configs
                                                          (and, with TQR_AUTO, the autotuner's tree
                                                          policies) */
int tqr_lstsq_batched(int32_t count, const int64_t *m, const int64_t *n, int64_t nrhs,
                      const double *const *A, const int64_t *lda, const double *const *B,
                      const int64_t *ldb, double *const *X, const int64_t *ldx, void *work,
                      size_t work_bytes, const tqr_opts *o, int32_t *info, hipStream_t stream);

/* Autotuner for a batch: runs tqr_lstsq_batched with every built (nb, ib)
 * configuration, times each on `stream` with HIP events, and writes the
 * fastest into *o (best_ms: NULL or its time).  With o->tree == TQR_AUTO it
 * also tries the kernel family and tree policy: the per-problem
 * critical-path tree with TT or TS kernels, and PlasmaTree with domains of
 * 4 or 8 tile rows and TS kernels; the fastest is written into o->kernels,
 * o->tree and o->param.  Otherwise the tree and family are the options'.
 * Synchronous.  The choice is cached per (shapes, nrhs, options), under
 * the options given and those chosen; a cached call returns at once with
 * *best_ms = -1.  work must hold tqr_lstsq_batched_work_size with
 * o->nb = 0 (which covers every configuration and policy tried).  X
 * receives the solutions of the last run. */
int tqr_autotune_batched(int32_t count, const int64_t *m, const int64_t *n, int64_t nrhs,
                         const double *const *A, const int64_t *lda, const double *const *B,
                         const int64_t *ldb, double *const *X, const int64_t *ldx, void *work,
                         size_t work_bytes, tqr_opts *o, float *best_ms, hipStream_t stream);

/* ------------------------------------------------ learned tree/nb selector
 *
 * A 3-layer perceptron (9 inputs, two hidden layers of 64 tanh units, one
 * output; FP32) predicts log(milliseconds) of a factorization from
 * features of (m, n, nb, tree, batch) (tqr_mlp_features).  It is trained on
 * the engine's own timings with the gradient and Adam kernels below and
 * registered with tqr_set_selector; TQR_AUTO then picks, per shape, the
 * (tree, nb) of smallest predicted time among the five trees and the built
 * tile sizes >= 64.  Without a registered network TQR_AUTO means GrASAP at
 * nb = 256.  (Project addition; the thesis selects trees by critical-path
 * analysis only.)  Parameters: W1 [64 x 9], b1 [64], W2 [64 x 64], b2 [64],
 * W3 [64], b3, contiguous FP32 in device memory. */
int32_t tqr_mlp_params(void);
int32_t tqr_mlp_features(void);
/* Feature vector (host) of one candidate: log2(m)/16, log2(n)/16,
 * log2(nb)/8, one-hot tree (FLAT, BINARY, FIBONACCI, GREEDY, GRASAP),
 * log2(batch)/10.  Returns 0, or -4 for a tree outside the five. */
int tqr_mlp_features_of(int64_t m, int64_t n, int32_t nb, int32_t tree, int32_t batch, float *out);
/* Device buffers: X [batch x 9] row-major, y / target [batch]. */
size_t tqr_mlp_work_size(int64_t batch);
int tqr_mlp_forward(const float *params, const float *X, int64_t batch, float *y, hipStream_t stream);
/* grad = d/dparams of mean((y - target)^2); loss (device float, may be
 * NULL) = that mean.  work: tqr_mlp_work_size(batch) bytes. */
int tqr_mlp_grad(const float *params, const float *X, const float *target, int64_t batch, float *grad,
                 float *loss, void *work, size_t work_bytes, hipStream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8), step >= 1; m1, m2 are
 * the caller's moment buffers (zero before step 1). */
int tqr_mlp_adam(float *params, const float *grad, float *m1, float *m2, int64_t step, float lr,
                 hipStream_t stream);
/* `epochs` full-batch Adam steps on (X, target); loss_hist (device, epochs
 * floats, may be NULL) receives the loss before each step. */
int tqr_mlp_fit(float *params, const float *X, const float *target, int64_t batch, int32_t epochs, float lr,
                float *loss_hist, void *work, size_t work_bytes, hipStream_t stream);
/* Registers (copies) a trained parameter vector from device memory; NULL
 * clears it.  Synchronous. */
int tqr_set_selector(const float *params);
/* The selector's choice for an m x n problem (batch: problems solved
 * together); host outputs.  Synchronous (runs the network on the current
 * device).  Falls back to GrASAP, 256, 32 without a registered network. */
int tqr_select(int64_t m, int64_t n, int32_t batch, int32_t *tree, int32_t *nb, int32_t *ib);

/* ----------------------------------------------- host-only list services */

/* Elimination list of `tree` (param: PlasmaTree BS / GrASAP i) for p x q
 * tiles (1 <= q <= p), as 1-based (i, piv, k) triples in list order.
 * Returns the list length, writing the triples only if cap >= length;
 * negative on bad arguments.  No GPU is touched. */
int64_t tqr_tree_list(int32_t tree, int32_t p, int32_t q, int32_t param, int32_t *i_out,
                      int32_t *piv_out, int32_t *k_out, int64_t cap);

/* Critical path, in units of nb^3/3 (table tab.kernels weights), of the
 * tiled algorithm given by the list and kernel family, on unbounded
 * processors; computed as the longest path of the task graph the executor
 * runs.  zero_t (p*q, row-major, may be NULL) receives the end time of the
 * kernel that zeroes each tile; counts (6, may be NULL) receives the number
 * of GEQRT, TSQRT, TTQRT, UNMQR, TSMQR, TTMQR tasks.  No GPU is touched. */
int64_t tqr_tree_cp(int32_t tree, int32_t p, int32_t q, int32_t param, int32_t kernels,
                    int64_t *zero_t, int64_t *counts);

/* Number of tasks and dependency edges of the executor's graph for the
 * given problem (factor only).  No GPU is touched. */
int tqr_graph_stats(int64_t m, int64_t n, const tqr_opts *o, int64_t *ntasks, int64_t *nedges);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * least-squares solve of tqr_lstsq (same arguments and results, same
 * kernels), with its workspace and task graphs placed in a device array of
 * TQR_NOALLOC_SCRATCH_BYTES that the library defines statically; every GPU
 * it runs on holds one such array until the process ends.  The call makes
 * no hipMalloc / hipFree and no allocating library call on the device (its
 * task graphs are built on the host, host memory, and cached per shape,
 * then copied into the array on `stream` at every call).  Every call on one
 * GPU uses that GPU's single array, so calls that overlap on one GPU (on
 * different streams, or from several threads) race; calls ordered on one
 * stream do not.  The array keeps the last call's contents; each call
 * resets what must start at zero (executor counters, refinement report)
 * on the stream.  Returns TQR_E_SCRATCH, and enqueues nothing, when the
 * workspace (tqr_lstsq_work_size) plus the task graphs exceed the array;
 * TQR_E_UNSUPPORTED for opts.tree = TQR_AUTO (the selector runs device
 * work); otherwise as tqr_lstsq. */
#define TQR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tqr_lstsq_noalloc(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                      int64_t ldb, double *X, int64_t ldx, const tqr_opts *o, int32_t *info,
                      hipStream_t stream);

/* ------------------------------------------------ double-complex tiled QR
 *
 * The tiled QR of a complex m x n matrix (m >= n), the thesis's "z"
 * workloads (chapter "QR Factorization", section "Experimental results"):
 * the same elimination lists, kernel families and task graph as the FP64
 * path, run by complex tile kernels (GEQRT, TSQRT, TTQRT, UNMQR, TSMQR,
 * TTMQR) in one persistent executor launch.  A: device memory, column-major,
 * interleaved (re, im) double pairs, lda >= m counted in complex entries;
 * on return (stream-ordered) the upper triangle of its first n rows holds
 * R, whose diagonal is real, and the other entries with the workspace W hold
 * the reflectors and their tau.  Reflector convention: for x = [alpha; x2],
 * beta = -sign(Re alpha) ||x||, tau = (beta - alpha) / beta,
 * v = [1; x2 / (alpha - beta)], H = I - tau v v^H, H^H x = beta e1 (tau = 0
 * when x2 = 0 and alpha is real).  Options from *o (NULL: defaults): nb 32
 * or 64 (default 64 when o is NULL), tree, param, kernels; ib, stripes,
 * priority and the precision fields are ignored (the ready order is the
 * static list order at nb 64, the dynamic queue at nb 32).  W:
 * tqr_zworkspace_size(m, n, nrhs, o)
 * bytes (nrhs: the widest B a later tqr_zapply_qh will take).  info: NULL
 * or a device int32 receiving 0 or TQR_INFO_TIMEOUT.  tqr_zapply_qh
 * overwrites B (m x nrhs, ldb >= m, complex) with Q^H B for a factorization
 * held in (A, W) with the same m, n and options. */
size_t tqr_zworkspace_size(int64_t m, int64_t n, int64_t nrhs, const tqr_opts *o);
int tqr_zfactor(int64_t m, int64_t n, void *A, int64_t lda, void *W, size_t w_bytes, const tqr_opts *o,
                int32_t *info, hipStream_t stream);
int tqr_zapply_qh(int64_t m, int64_t n, const void *A, int64_t lda, void *W, size_t w_bytes, int64_t nrhs,
                  void *B, int64_t ldb, const tqr_opts *o, int32_t *info, hipStream_t stream);

/* ------------------------------------------------ tile Cholesky inversion
 *
 * A^{-1} of a symmetric positive definite n x n matrix, in place, by the
 * thesis's tile algorithm (chapter "Cholesky Inversion", algorithm
 * alg:InPlace): step 1 the tile Cholesky factorization A = L L^T, step 2
 * W = L^{-1}, step 3 A^{-1} = W^T W, all three as one task graph (steps
 * pipelined) run by one persistent executor launch.  A: device,
 * column-major, lda >= n; only its lower triangle is read, and on return
 * (stream-ordered) the lower triangle holds that of A^{-1}; the strict upper
 * triangle is not touched.  nb: tile size, 32 or 64 (n need not be a
 * multiple).  variant: TQR_CHOLINV_INPLACE (the algorithm as printed) or
 * TQR_CHOLINV_RENAMED (array renaming, section "Algorithmic study": steps 2
 * and 3 read L and L^{-1} from copies in `work`, which removes their
 * anti-dependences and shortens the critical path), optionally |
 * TQR_CHOLINV_UUU (every innermost GEMM loop upward; the default UDU runs
 * step 2's downward, which the same section shows is shorter).  work:
 * tqr_cholinv_work_size bytes of device memory (executor state, and the
 * copies for the renamed variant).  info: NULL or a device int32 receiving
 * 0, k > 0 when the leading minor of order k is not positive definite (the
 * result is then undefined), or TQR_INFO_TIMEOUT.  Returns 0 or -i for an
 * illegal i-th argument / a TQR_E_* code. */
enum { TQR_CHOLINV_INPLACE = 0, TQR_CHOLINV_RENAMED = 1, TQR_CHOLINV_UUU = 2 };
size_t tqr_cholinv_work_size(int64_t n, int32_t nb, int32_t variant);
int tqr_cholinv(int64_t n, double *A, int64_t lda, int32_t nb, int32_t variant, void *work, size_t work_bytes,
                int32_t *info, hipStream_t stream);

/* Task count and critical path of the inversion's graph for t x t tiles,
 * in tasks (table table:criticalpath counts tasks) and weighted (units of
 * nb^3/3).  Host only. */
int tqr_cholinv_graph_stats(int32_t t, int32_t variant, int64_t *ntasks, double *cp_tasks, double *cp_weighted);

/* Bounded-processor schedule analysis of the factorization's task graph
 * for the problem and options given (the graph tqr_factor runs: tree,
 * kernel family, update stripes; weights of table tab.kernels divided
 * among a tile's stripes), on P processors, from the thesis's chapters
 * "Scheduling of Cholesky Factorization" (section "ALAP Derived Performance
 * Bound", equation eqn:alapbound) and "Scheduling of QR Factorization"
 * (section "Optimality", table tab:5x5_optimal).  out[5] receives, in units
 * of nb^3/3: the critical path; the total work T_seq; the lost area LA_P
 * of P processors at the end of the as-late-as-possible execution on
 * unbounded processors; the ALAP derived bound max(cp, (T_seq + LA_P)/P),
 * a lower bound on any schedule's length on P processors; and the length of
 * the critical-path list schedule on P processors (an idle processor takes
 * the ready task of largest bottom level; ties to the task ready first,
 * then to the later one in list order).  Host only: no GPU is touched.
 * Returns 0, or -i for an illegal i-th argument. */
int tqr_schedule_bounds(int64_t m, int64_t n, const tqr_opts *o, int32_t P, double *out);

const char *tqr_strerror(int code);

/* Number of workgroups of the persistent executor launch for the tile
 * configuration of *o (NULL: defaults) on the current device: the number
 * of tasks that can run at once (compute units x resident workgroups per
 * unit).  Negative on unsupported options or a failed HIP query. */
int tqr_executor_grid(const tqr_opts *o);

/* ---------------------------------------------------------- diagnostics */

/* Debug only, not thread-safe: while buf is non-NULL every executor launch
 * records, for each task t < cap, four int64 at buf + 4t: start and end
 * (device wall clock, hipDeviceAttributeWallClockRate kHz), the workgroup
 * and the hardware CU id that ran it.  buf is a device buffer owned by the
 * caller.  Pass NULL to stop. */
void tqr_debug_trace(int64_t *buf, int64_t cap);

/* Rate of the device wall clock used by the trace stamps and the watchdog
 * (hipDeviceAttributeWallClockRate of the current device), in kHz, or a
 * negative TQR_E_* code. */
int64_t tqr_wallclock_khz(void);

/* Debug only: the executor's watchdog limit, in device wall-clock ticks
 * (hipDeviceAttributeWallClockRate kHz), for every later launch: a
 * workgroup that waits longer than this for its queue slot to hold a ready
 * task sets the abort flag, every workgroup then leaves the executor and
 * info receives TQR_INFO_TIMEOUT (the results are then undefined).  0
 * restores the default of 30 seconds.  A tiny limit forces the watchdog
 * path from the host (failure-handling tests); every kernel still exits. */
void tqr_debug_spin_limit(int64_t ticks);

/* Diagnostics: with timing enabled, every executor launch is bracketed by a
 * pair of HIP events recorded on the launch's stream (the executor kernel
 * alone, not the copies or resets around it).  tqr_debug_timing(1) starts a
 * new measurement (dropping earlier events), tqr_debug_timing(0) stops.
 * tqr_debug_timing_read waits for the recorded launches and returns their
 * summed duration in milliseconds and their number.  Not thread-safe with
 * respect to concurrent launches on several streams. */
void tqr_debug_timing(int32_t enable);
int tqr_debug_timing_read(double *ms_total, int64_t *launches);

/* Debug only: the executor's task table for a plan (kind 0 factor, 1 apply
 * with nrhs columns, 2 solve, 3 the least-squares graph of tqr_lstsq; 6 the
 * Cholesky inversion of order m = n with tile size o->nb and variant
 * o->param, its tasks' i, piv, k, j being the tile indices i, i, k, j) as 8
 * int32 per task: kind, i, piv, k, j,
 * stripe, number of successors, number of predecessors.  Returns the task
 * count (tasks written only if cap >= count). */
int tqr_debug_graph(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o,
                    int32_t *tasks, int64_t cap);

/* Debug only: successor lists (CSR) of a plan (kind and nrhs as for
 * tqr_debug_graph); off has ntasks+1 entries, succ cap entries.  Returns the
 * number of edges, or a negative value (bad arguments, cap too small). */
int tqr_debug_succ(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o, int32_t *off,
                   int32_t *succ, int64_t cap);

/* Debug only: the initially ready tasks of a plan (kind and nrhs as for
 * tqr_debug_graph) in queue order: with TQR_PRIO_STATIC every task, in the
 * order the executor hands them out.  Returns their number, or a negative
 * value (bad arguments, cap too small). */
int tqr_debug_ready(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o, int32_t *ready,
                    int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* TQR_H */
