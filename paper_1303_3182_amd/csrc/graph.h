// Host-side scheduling layer: elimination lists and the task graph that the
// device executor runs.
#pragma once
#include <cstdint>
#include <vector>

#include "tqr_types.h"

namespace tqr {

// One elimination elim(i, piv, k) of algorithm alg.QR, 0-based.
struct Elim {
  int i, piv, k;
};

enum TreeId { TREE_FLAT = 0, TREE_BINARY = 1, TREE_FIBONACCI = 2, TREE_GREEDY = 3,
              TREE_GRASAP = 4, TREE_PLASMA = 5, TREE_ASAP = 6 };
enum KernelFamily { FAM_TT = 0, FAM_HYBRID = 1 };

// Elimination list of a tree for p x q tiles (p >= q >= 1); param is the
// PlasmaTree domain size or the i of GrASAP(i).  Empty on bad input.
std::vector<Elim> make_list(int tree, int p, int q, int param);

// Task weights of table tab.kernels (unit nb^3/3); the solve kernels are
// weighted by their flops in the same unit.
double kind_weight(int kind);

// Task graph of the tiled algorithm.
//
// The elimination list is expanded, in list order, into kernels following
// algorithm alg.elimTR (TT family) or the hybrid rule (a row is
// triangularised at its first use as a pivot, a square tile is zeroed with
// TSQRT/TSMQR as in algorithm alg.elimSQ, a triangle with TTQRT/TTMQR).
// Dependencies are derived from the data each kernel reads and writes, in
// that sequential order (read-after-write, write-after-read,
// write-after-write), over these data items:
//   X(i,j,s)  stripe s of tile (i,j) as an update target,
//   U(i,k)    the upper triangle of a factored tile (R, or TT reflectors),
//   L(i,k)    its strict lower part (GEQRT reflectors),
//   TG(i,k)   GEQRT's T, TK(i,k) the T of the kernel that zeroes (i,k).
// Splitting a tile update into stripes is exact: Q^T acts column by column.
struct GraphSpec {
  int p = 1, q = 1;      // tile rows / tile columns of A
  int family = FAM_TT;
  int stripes = 1;       // update tasks per target tile of A
  int nbcols = 0;        // tile columns of B (right-hand sides)
  int stripes_b = 1;     // update tasks per target tile of B
  bool panels = true;    // emit the factor kernels (and A-column updates)
  bool b_updates = false;  // emit updates of the B columns
  bool solve_t = false;  // emit the forward substitution R^T Z = B (after the above)
  bool solve = false;    // emit the back-substitution R X = B (after the above)
};

struct Graph {
  std::vector<Task> tasks;                  // in a topological (list) order
  std::vector<std::vector<int32_t>> preds;  // deduplicated predecessors
  std::vector<double> weight;               // per task, unit nb^3/3
  std::vector<double> finish;               // earliest finish, unbounded processors
  // filled by finalize():
  std::vector<int32_t> succ_off, succ, indeg0, ready0, order;
  std::vector<double> bottom;  // longest path from the task to an exit, incl. itself
  int64_t nedges = 0;
  double cp = 0.0;
  // set by static_list_order(): ready0 lists every task, in the order the
  // executor hands them out
  bool static_order = false;
};

// Builds the graph of `list` under `spec`.  zero_t / geqrt_t, when given
// (p*q, row-major, 0-based), receive the earliest finish of the kernel that
// zeroes / triangularises each tile.
Graph build_graph(const std::vector<Elim> &list, const GraphSpec &spec,
                  std::vector<double> *zero_t = nullptr, std::vector<double> *geqrt_t = nullptr);

// Successor lists, dependency counts, bottom levels and the initial ready
// order (highest bottom level first when `priority`, else list order).
void finalize(Graph &g, bool priority);

// Simulates the critical-path list schedule of a finalized QR graph on P
// workgroups with estimated GPU task durations at tile size nb (the
// tab.kernels weights scaled per kernel by task durations measured on
// MI355X at nb 64, 128 and 256: the panel kernels' Householder steps are
// latency-bound, so their time per flop is 2.5 to 4 times the updates'; a
// free workgroup starts the ready task of largest bottom level under these
// durations, ties to the earlier ready time, then the lower index) and sets
// ready0 to every task in simulated start order, with static_order.  Predecessors always start
// before their successors in this order.  Returns the simulated makespan
// (estimated microseconds).
double static_list_order(Graph &g, int P, int nb, bool complex_kernels = false);

// Task graph of the tile Cholesky inversion of t x t tiles (thesis chapter
// "Cholesky Inversion", algorithm alg:InPlace: step 1 the tile Cholesky
// factorization, step 2 the inversion of L, step 3 the product
// L^{-T} L^{-1}), in the algorithm's loop order with the steps pipelined
// (every task waits only for the data it needs).  Items: tile (i,j) of the
// lower triangle, updated in place.  inplace = false is the variant with
// array renaming: the last writer of a tile in step 1 (step 2) also writes a
// copy of it, and step 2 (step 3) reads L (L^{-1}) from those copies, so
// those reads carry no anti-dependences.  udu: the innermost loop of step 2
// runs downward (loop order UDU, the shorter critical path), else upward
// (UUU).  Weights in units of nb^3/3 (POTRF, TRTRI, LAUUM 1; TRSM, SYRK,
// TRMM 3; GEMM 6); unit_weights counts tasks instead.
Graph build_cholinv_graph(int t, bool inplace, bool udu, bool unit_weights = false);

// Bounded-processor analysis of a finalized graph, in its weight unit
// (thesis chapters "Scheduling of Cholesky Factorization", section "ALAP
// Derived Performance Bound", equation eqn:alapbound, and "Scheduling of QR
// Factorization", section "Optimality"):
//   alap_lost_area: every task placed as late as possible on unbounded
//     processors (start = cp - bottom level); the idle area of P
//     processors over the tail of that placement in which it never uses
//     more than P of them;
//   alap_bound: max(cp, (total weight + lost area) / P), a lower bound on
//     the makespan of any schedule on P processors;
//   list_makespan: the critical-path list schedule on P processors (an idle
//     processor starts the ready task of largest bottom level; ties to the
//     earliest ready, then the latest in list order).
double alap_lost_area(const Graph &g, int P);
double alap_bound(const Graph &g, int P);
double list_makespan(const Graph &g, int P);

// Host-side check that the graph is acyclic and that dependency counts
// match (a Kahn pass over the successor lists).
bool validate(const Graph &g);

}  // namespace tqr
