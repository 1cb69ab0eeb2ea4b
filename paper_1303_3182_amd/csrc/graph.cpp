// Elimination lists (thesis section "Critical paths") and the task graph of
// the tiled algorithm (sections "Kernels", "Execution schemes").
#include "graph.h"

#include <algorithm>
#include <cstdlib>
#include <functional>
#include <queue>
#include <utility>

namespace tqr {

// ----------------------------------------------------------------- weights
double kind_weight(int kind) {
  switch (kind) {
    case K_GEQRT: return 4.0;
    case K_TSQRT: return 6.0;
    case K_TTQRT: return 2.0;
    case K_UNMQR: return 6.0;
    case K_TSMQR: return 12.0;
    case K_TTMQR: return 6.0;
    case K_TRSM: return 1.0;  // nb^3 flops
    case K_GEMM: return 6.0;  // 2 nb^3 flops
    case K_TRSMT: return 1.0;
    case K_GEMMT: return 6.0;
    default: return 0.0;
  }
}

// ------------------------------------------------------------ graph build
namespace {

struct ItemState {
  int32_t writer = -1;
  std::vector<int32_t> readers;
};

class Builder {
 public:
  Builder(const GraphSpec &s, bool keep_structure)
      : spec_(s), keep_(keep_structure), p_(s.p), q_(s.q), qt_(s.q + s.nbcols),
        tri_((size_t)s.p * s.q, 0), zero_((size_t)s.p * s.q, 0.0), geqrt_((size_t)s.p * s.q, 0.0) {
    const int smax = std::max(s.stripes, s.stripes_b);
    smax_ = smax;
    x_.resize((size_t)p_ * qt_ * smax);
    u_.resize((size_t)p_ * q_);
    l_.resize((size_t)p_ * q_);
    tg_.resize((size_t)p_ * q_);
    tk_.resize((size_t)p_ * q_);
  }

  Graph &graph() { return g_; }
  const std::vector<double> &zero_times() const { return zero_; }
  const std::vector<double> &geqrt_times() const { return geqrt_; }

  // Kernels that the first column needs before any elimination (TT only:
  // algorithm alg.elimTR with k = 0 triangularises every tile of column 1).
  void start() {
    if (solve_only()) return;
    if (spec_.family == FAM_TT)
      for (int i = 0; i < p_; i++) factor_row(i, 0);
  }

  void elim(const Elim &e) {
    const int i = e.i, piv = e.piv, k = e.k;
    if (spec_.family == FAM_TT) {
      zero(K_TTQRT, K_TTMQR, i, piv, k);
      if (k + 1 < q_) factor_row(i, k + 1);
    } else {
      if (!tri_[idx(piv, k)]) factor_row(piv, k);
      if (tri_[idx(i, k)])
        zero(K_TTQRT, K_TTMQR, i, piv, k);
      else
        zero(K_TSQRT, K_TSMQR, i, piv, k);
    }
  }

  void end() {
    if (solve_only()) return;
    // The last diagonal tile of a square tile matrix is never a pivot in
    // the hybrid family; it still has to be triangularised.
    if (spec_.family == FAM_HYBRID && p_ == q_ && !tri_[idx(q_ - 1, q_ - 1)])
      factor_row(q_ - 1, q_ - 1);
  }

  // Back-substitution R X = B over the tile columns of B: for k = q-1..0,
  // X(k) = R(k,k)^{-1} B(k), then B(i) -= R(i,k) X(k) for i < k.  R(k,k)
  // is the triangle item of tile (k,k); R(i,k), i < k, is the last state of
  // the update target tile (i,k) (every stripe), so after a factorization
  // in the same graph these tasks wait for exactly the kernels that
  // finish those tiles.
  void solve() {
    for (int jb = 0; jb < spec_.nbcols; jb++)
      for (int s = 0; s < spec_.stripes_b; s++)
        for (int k = q_ - 1; k >= 0; k--) {
          emit(K_TRSM, k, k, k, q_ + jb, s, {&u_[idx(k, k)]}, {xitem(k, q_ + jb, s)});
          for (int i = k - 1; i >= 0; i--) {
            std::vector<ItemState *> rd = {xitem(k, q_ + jb, s)};
            for (int sa = 0; sa < spec_.stripes; sa++) rd.push_back(xitem(i, k, sa));
            emit(K_GEMM, i, i, k, q_ + jb, s, rd, {xitem(i, q_ + jb, s)});
          }
        }
  }

  // Forward substitution R^T Z = B (R^T lower triangular): for k = 0..q-1,
  // Z(k) = R(k,k)^{-T} B(k), then B(i) -= R(k,i)^T Z(k) for i > k.
  void solve_t() {
    for (int jb = 0; jb < spec_.nbcols; jb++)
      for (int s = 0; s < spec_.stripes_b; s++)
        for (int k = 0; k < q_; k++) {
          emit(K_TRSMT, k, k, k, q_ + jb, s, {&u_[idx(k, k)]}, {xitem(k, q_ + jb, s)});
          for (int i = k + 1; i < q_; i++) {
            std::vector<ItemState *> rd = {xitem(k, q_ + jb, s)};
            for (int sa = 0; sa < spec_.stripes; sa++) rd.push_back(xitem(k, i, sa));
            emit(K_GEMMT, i, i, k, q_ + jb, s, rd, {xitem(i, q_ + jb, s)});
          }
        }
  }

 private:
  bool solve_only() const { return (spec_.solve || spec_.solve_t) && !spec_.panels && !spec_.b_updates; }
  size_t idx(int i, int k) const { return (size_t)i * q_ + k; }
  ItemState *xitem(int i, int j, int s) { return &x_[((size_t)i * qt_ + j) * smax_ + s]; }
  int stripes_of(int j) const { return j < q_ ? spec_.stripes : spec_.stripes_b; }

  // Target columns of the updates that follow a factor kernel of column k.
  template <typename F>
  void for_targets(int k, F f) {
    if (spec_.panels)
      for (int j = k + 1; j < q_; j++) f(j);
    if (spec_.b_updates)
      for (int j = q_; j < qt_; j++) f(j);
  }

  void factor_row(int i, int k) {
    if (spec_.panels) {
      std::vector<ItemState *> w = {&u_[idx(i, k)], &l_[idx(i, k)], &tg_[idx(i, k)]};
      for (int s = 0; s < spec_.stripes; s++) w.push_back(xitem(i, k, s));
      geqrt_[idx(i, k)] = emit(K_GEQRT, i, i, k, k, 0, {}, w);
    }
    tri_[idx(i, k)] = 1;
    for_targets(k, [&](int j) {
      for (int s = 0; s < stripes_of(j); s++)
        emit(K_UNMQR, i, i, k, j, s, {&l_[idx(i, k)], &tg_[idx(i, k)]}, {xitem(i, j, s)});
    });
  }

  void zero(int fk, int uk, int i, int piv, int k) {
    if (spec_.panels) {
      std::vector<ItemState *> w = {&u_[idx(piv, k)], &u_[idx(i, k)], &tk_[idx(i, k)]};
      if (fk == K_TSQRT) {
        w.push_back(&l_[idx(i, k)]);
        for (int s = 0; s < spec_.stripes; s++) w.push_back(xitem(i, k, s));
      }
      zero_[idx(i, k)] = emit(fk, i, piv, k, k, 0, {}, w);
    }
    for_targets(k, [&](int j) {
      for (int s = 0; s < stripes_of(j); s++) {
        std::vector<ItemState *> r = {&u_[idx(i, k)], &tk_[idx(i, k)]};
        if (uk == K_TSMQR) r.push_back(&l_[idx(i, k)]);
        emit(uk, i, piv, k, j, s, r, {xitem(piv, j, s), xitem(i, j, s)});
      }
    });
  }

  // Appends one task; `rd` are read-only items, `wr` read-write items.
  // Returns the task's earliest finish.
  double emit(int kind, int i, int piv, int k, int j, int s, std::vector<ItemState *> rd,
              std::vector<ItemState *> wr) {
    const int32_t id = (int32_t)g_.finish.size();
    std::vector<int32_t> pr;
    for (ItemState *it : rd)
      if (it->writer >= 0) pr.push_back(it->writer);
    for (ItemState *it : wr) {
      if (it->writer >= 0) pr.push_back(it->writer);
      for (int32_t r : it->readers) pr.push_back(r);
    }
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    double w = kind_weight(kind);
    if (kind >= K_UNMQR && kind <= K_TTMQR) w /= stripes_of(j);
    if (kind == K_TRSM || kind == K_GEMM || kind == K_TRSMT || kind == K_GEMMT) w /= spec_.stripes_b;
    double start = 0.0;
    for (int32_t x : pr) start = std::max(start, g_.finish[x]);
    const double fin = start + w;
    g_.finish.push_back(fin);
    g_.cp = std::max(g_.cp, fin);
    g_.nedges += (int64_t)pr.size();
    for (ItemState *it : rd) it->readers.push_back(id);
    for (ItemState *it : wr) {
      it->writer = id;
      it->readers.clear();
    }
    if (keep_) {
      Task t{};
      t.kind = kind;
      t.i = i;
      t.piv = piv;
      t.k = k;
      t.j = j;
      t.stripe = s;
      g_.tasks.push_back(t);
      g_.preds.push_back(std::move(pr));
      g_.weight.push_back(w);
    }
    return fin;
  }

  GraphSpec spec_;
  bool keep_;
  int p_, q_, qt_, smax_ = 1;
  std::vector<ItemState> x_, u_, l_, tg_, tk_;
  std::vector<char> tri_;
  std::vector<double> zero_, geqrt_;
  Graph g_;
};

}  // namespace

// ---------------------------------------------------------------- lists

// Sameh-Kuck / FlatTree: the diagonal row zeroes every tile below it.
static void list_flat(int p, int q, std::vector<Elim> &out) {
  for (int k = 0; k < std::min(p, q); k++)
    for (int i = k + 1; i < p; i++) out.push_back({i, k, k});
}

// BinaryTree: pairwise reduction of rows k..p-1 anchored at row k; at
// distance h the row k + d (d an odd multiple of h) is zeroed by k + d - h.
static void list_binary(int p, int q, std::vector<Elim> &out) {
  for (int k = 0; k < std::min(p, q); k++) {
    const int rows = p - k;
    for (int h = 1; h < rows; h <<= 1)
      for (int d = h; d < rows; d += h << 1) out.push_back({k + d, k + d - h, k});
  }
}

// Fibonacci scheme of order 1 (Modi-Clarke): in column k the row at
// relative position r = i - k + 1 (1-based) belongs to group y(r), the least
// y with r <= y(y+1)/2 + 1.  Groups are zeroed from the bottom (largest y)
// up; a group of z consecutive rows is zeroed by the z rows just above it.
static void list_fibonacci(int p, int q, std::vector<Elim> &out) {
  for (int k = 0; k < std::min(p, q); k++) {
    std::vector<std::vector<int>> groups;  // groups[y-1] = rows (ascending)
    int y = 1;
    for (int i = k + 1; i < p; i++) {
      const int r = i - k + 1;
      while (r > y * (y + 1) / 2 + 1) y++;
      if ((int)groups.size() < y) groups.resize(y);
      groups[y - 1].push_back(i);
    }
    for (int gi = (int)groups.size() - 1; gi >= 0; gi--) {
      const int z = (int)groups[gi].size();
      for (int i : groups[gi]) out.push_back({i, i - z, k});
    }
  }
}

// Greedy (algorithm alg.tiled-greedy).  Per column j the counters nT (tiles
// triangularised) and nZ (tiles zeroed) grow from the bottom row up.  At
// each step, columns are visited from right to left; column j can
// triangularise the tiles zeroed in column j-1 at earlier steps, and zeroes
// half of its triangular-but-live tiles, the bottom ones, each with the
// row `half` places above.  The number of new zeros uses the updated nT of
// this step.
static void list_greedy(int p, int q, std::vector<Elim> &out) {
  const int last = std::min(q, p - 1) - 1;  // last column with eliminations
  if (last < 0) return;
  std::vector<int> nT(q, 0), nZ(q, 0);
  while (nZ[last] < p - 1 - last) {
    for (int j = q - 1; j >= 0; j--) {
      const int t = (j == 0) ? p : nZ[j - 1];
      const int half = (t - nZ[j]) / 2;
      for (int a = 0; a < half; a++) {
        const int row = p - 1 - nZ[j] - a;
        out.push_back({row, row - half, j});
      }
      nT[j] = t;
      nZ[j] += half;
    }
  }
}

// PlasmaTree(BS): domains of BS consecutive rows starting at the diagonal
// row (the last one truncated); a flat tree inside each domain, then a
// binary tree across the domain heads.
static void list_plasma(int p, int q, int bs, std::vector<Elim> &out) {
  if (bs < 1) bs = 1;
  for (int k = 0; k < std::min(p, q); k++) {
    for (int h = k; h < p; h += bs)
      for (int i = h + 1; i < std::min(p, h + bs); i++) out.push_back({i, h, k});
    const int heads = (p - 1 - k) / bs + 1;
    for (int h = 1; h < heads; h <<= 1)
      for (int d = h; d < heads; d += h << 1) out.push_back({k + d * bs, k + (d - h) * bs, k});
  }
}

// ASAP on one column (definition def.optiter with w = TTQRT's weight): rows
// become available when their GEQRT ends; whenever at least two available
// rows are idle, the bottom 2s of them are paired, the upper s zeroing the
// lower s in order; a pivot is busy for one TTQRT.
static void asap_column(int k, const std::vector<double> &ready, std::vector<Elim> &out) {
  const int p = (int)ready.size();
  const double w = kind_weight(K_TTQRT);
  std::vector<double> busy(p, 0.0);
  std::vector<char> live(p, 0);
  int nlive = 0;
  for (int r = k; r < p; r++) {
    live[r] = 1;
    nlive++;
  }
  double t = 1e300;
  for (int r = k; r < p; r++) t = std::min(t, ready[r]);
  std::vector<int> av;
  while (nlive > 1) {
    av.clear();
    for (int r = k; r < p; r++)
      if (live[r] && ready[r] <= t && busy[r] <= t) av.push_back(r);
    const int s = (int)av.size() / 2;
    const int base = (int)av.size() - 2 * s;
    for (int a = 0; a < s; a++) {
      const int piv = av[base + a], row = av[base + s + a];
      out.push_back({row, piv, k});
      busy[piv] = t + w;
      live[row] = 0;
      nlive--;
    }
    double nt = 1e300;
    for (int r = k; r < p; r++) {
      if (!live[r]) continue;
      if (ready[r] > t) nt = std::min(nt, ready[r]);
      if (busy[r] > t) nt = std::min(nt, busy[r]);
    }
    if (nt >= 1e300) break;
    t = nt;
  }
}

// GrASAP(ia): Greedy on columns 0..q-ia-1, ASAP on the last ia columns
// using the tiled GEQRT end times of the list built so far (definition
// def.grasap).
void asap_columns(int p, int q, int ia, std::vector<Elim> &out) {
  std::vector<Elim> greedy;
  list_greedy(p, q, greedy);
  GraphSpec spec;
  spec.p = p;
  spec.q = q;
  Builder b(spec, false);
  b.start();
  for (const Elim &e : greedy)
    if (e.k < q - ia) {
      out.push_back(e);
      b.elim(e);
    }
  for (int k = std::max(0, q - ia); k < std::min(q, p - 1); k++) {
    std::vector<double> ready(p, 0.0);
    for (int r = k; r < p; r++) ready[r] = b.geqrt_times()[(size_t)r * q + k];
    const size_t before = out.size();
    asap_column(k, ready, out);
    for (size_t e = before; e < out.size(); e++) b.elim(out[e]);
  }
}

std::vector<Elim> make_list(int tree, int p, int q, int param) {
  std::vector<Elim> out;
  if (p < 1 || q < 1 || q > p) return out;
  switch (tree) {
    case TREE_FLAT: list_flat(p, q, out); break;
    case TREE_BINARY: list_binary(p, q, out); break;
    case TREE_FIBONACCI: list_fibonacci(p, q, out); break;
    case TREE_GREEDY: list_greedy(p, q, out); break;
    case TREE_GRASAP: asap_columns(p, q, param < 1 ? 1 : std::min(param, q), out); break;
    case TREE_PLASMA: list_plasma(p, q, param, out); break;
    case TREE_ASAP: asap_columns(p, q, q, out); break;
    default: break;
  }
  return out;
}

Graph build_graph(const std::vector<Elim> &list, const GraphSpec &spec, std::vector<double> *zero_t,
                  std::vector<double> *geqrt_t) {
  Builder b(spec, true);
  if (spec.panels || spec.b_updates) {
    b.start();
    for (const Elim &e : list) b.elim(e);
    b.end();
  }
  if (spec.solve_t) b.solve_t();
  if (spec.solve) b.solve();
  if (zero_t) *zero_t = b.zero_times();
  if (geqrt_t) *geqrt_t = b.geqrt_times();
  return std::move(b.graph());
}

void finalize(Graph &g, bool priority) {
  const int n = (int)g.tasks.size();
  std::vector<std::vector<int32_t>> succ(n);
  for (int t = 0; t < n; t++)
    for (int32_t pr : g.preds[t]) succ[pr].push_back(t);
  g.bottom.assign(n, 0.0);
  for (int t = n - 1; t >= 0; t--) {  // list order is topological
    double m = 0.0;
    for (int32_t s : succ[t]) m = std::max(m, g.bottom[s]);
    g.bottom[t] = g.weight[t] + m;
  }
  g.succ_off.assign(n + 1, 0);
  g.succ.clear();
  g.succ.reserve(g.nedges);
  g.indeg0.assign(n, 0);
  for (int t = 0; t < n; t++) {
    std::vector<int32_t> &s = succ[t];
    if (priority)
      std::stable_sort(s.begin(), s.end(), [&](int32_t a, int32_t b) { return g.bottom[a] > g.bottom[b]; });
    g.succ_off[t] = (int32_t)g.succ.size();
    for (int32_t x : s) g.succ.push_back(x);
    g.indeg0[t] = (int32_t)g.preds[t].size();
  }
  g.succ_off[n] = (int32_t)g.succ.size();
  g.ready0.clear();
  for (int t = 0; t < n; t++)
    if (g.indeg0[t] == 0) g.ready0.push_back(t);
  if (priority)
    std::stable_sort(g.ready0.begin(), g.ready0.end(),
                     [&](int32_t a, int32_t b) { return g.bottom[a] > g.bottom[b]; });
  g.order.resize(n);
  for (int t = 0; t < n; t++) g.order[t] = t;
}

namespace {
// Estimated GPU duration (microseconds) per unit of tab.kernels weight, from
// the mean task durations of traced least-squares launches on MI355X (TRSM
// and GEMM with one right-hand side), per tile size; nb 32 takes nb 64's.
double gpu_cost_per_unit(int kind, int nb) {
  //                              GEQRT  TSQRT  TTQRT  UNMQR  TSMQR  TTMQR  TRSM  GEMM
  static const double c64[8] = {17.8, 13.5, 37.5, 4.4, 2.2, 3.8, 9.0, 1.0};
  static const double c128[8] = {37.0, 31.0, 74.0, 8.3, 6.0, 9.6, 20.0, 1.7};
  static const double c256[8] = {134.0, 126.0, 247.0, 54.0, 41.0, 62.0, 42.0, 3.6};
  const double *c = nb >= 256 ? c256 : (nb >= 128 ? c128 : c64);
  switch (kind) {
    case K_GEQRT: return c[0];
    case K_TSQRT: return c[1];
    case K_TTQRT: return c[2];
    case K_UNMQR: return c[3];
    case K_TSMQR: return c[4];
    case K_TTMQR: return c[5];
    case K_TRSM:
    case K_TRSMT: return c[6];
    case K_GEMM:
    case K_GEMMT: return c[7];
    default: return 1.0;
  }
}
// The double-complex kernels at nb 64 (one reflector at a time on the
// vector units, 512 threads per workgroup): microseconds per unit of
// tab.kernels weight from a traced 8192 x 2048 factorization.
double gpu_cost_per_unit_z(int kind) {
  switch (kind) {
    case K_GEQRT: return 26.3;
    case K_TSQRT: return 23.3;
    case K_TTQRT: return 49.6;
    case K_UNMQR: return 6.1;
    case K_TSMQR: return 3.5;
    case K_TTMQR: return 6.6;
    default: return 1.0;
  }
}
}  // namespace

double static_list_order(Graph &g, int P, int nb, bool complex_kernels) {
  const int n = (int)g.tasks.size();
  P = std::max(P, 1);
  std::vector<double> w(n), bot(n, 0.0);
  for (int t = 0; t < n; t++)
    w[t] = g.weight[t] * (complex_kernels ? gpu_cost_per_unit_z(g.tasks[t].kind) : gpu_cost_per_unit(g.tasks[t].kind, nb));
  for (int t = n - 1; t >= 0; t--) {  // list order is topological
    double m = 0.0;
    for (int e = g.succ_off[t]; e < g.succ_off[t + 1]; e++) m = std::max(m, bot[g.succ[e]]);
    bot[t] = w[t] + m;
  }
  struct Ready {
    double pri, at;
    int32_t id;
    bool operator<(const Ready &o) const {  // max-heap: the "largest" starts first
      if (pri != o.pri) return pri < o.pri;
      if (at != o.at) return at > o.at;
      return id > o.id;
    }
  };
  std::priority_queue<Ready> ready;
  using Run = std::pair<double, int32_t>;  // (end, id), earliest end first
  std::priority_queue<Run, std::vector<Run>, std::greater<Run>> running;
  std::vector<int32_t> deg(g.indeg0.begin(), g.indeg0.end());
  for (int t = 0; t < n; t++)
    if (deg[t] == 0) ready.push({bot[t], 0.0, t});
  std::vector<int32_t> order;
  order.reserve(n);
  double now = 0.0, makespan = 0.0;
  int idle = P;
  while ((int)order.size() < n || !running.empty()) {
    while (idle > 0 && !ready.empty()) {
      const Ready r = ready.top();
      ready.pop();
      order.push_back(r.id);
      running.push({now + w[r.id], r.id});
      idle--;
    }
    if (running.empty()) break;  // (a cycle would stop here; validate() rejects those)
    now = running.top().first;
    while (!running.empty() && running.top().first == now) {
      const int32_t t = running.top().second;
      running.pop();
      idle++;
      makespan = std::max(makespan, now);
      for (int e = g.succ_off[t]; e < g.succ_off[t + 1]; e++)
        if (--deg[g.succ[e]] == 0) ready.push({bot[g.succ[e]], now, g.succ[e]});
    }
  }
  g.ready0 = order;
  g.static_order = true;
  return makespan;
}

// --------------------------------------------- tile Cholesky inversion
Graph build_cholinv_graph(int t, bool inplace, bool udu, bool unit_weights) {
  Graph g;
  std::vector<ItemState> tiles((size_t)t * t), l0((size_t)t * t), w0((size_t)t * t);
  auto A = [&](int i, int j) { return &tiles[(size_t)i * t + j]; };
  auto L0 = [&](int i, int j) { return &l0[(size_t)i * t + j]; };
  auto W0 = [&](int i, int j) { return &w0[(size_t)i * t + j]; };
  auto weight = [&](int kind) -> double {
    if (unit_weights) return 1.0;
    switch (kind) {
      case K_POTRF: case K_TRTRI: case K_LAUUM: return 1.0;
      case K_CGEMM: case K_IGEMM: case K_PGEMM: return 6.0;
      default: return 3.0;  // TRSM, SYRK, TRMM
    }
  };
  auto emit = [&](int kind, int i, int j, int k, std::vector<ItemState *> rd, std::vector<ItemState *> wr) {
    const int32_t id = (int32_t)g.tasks.size();
    std::vector<int32_t> pr;
    for (ItemState *it : rd)
      if (it->writer >= 0) pr.push_back(it->writer);
    for (ItemState *it : wr) {
      if (it->writer >= 0) pr.push_back(it->writer);
      for (int32_t r : it->readers) pr.push_back(r);
    }
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    const double w = weight(kind);
    double start = 0.0;
    for (int32_t x : pr) start = std::max(start, g.finish[x]);
    g.finish.push_back(start + w);
    g.cp = std::max(g.cp, start + w);
    g.nedges += (int64_t)pr.size();
    for (ItemState *it : rd) it->readers.push_back(id);
    for (ItemState *it : wr) {
      it->writer = id;
      it->readers.clear();
    }
    Task tk{};
    tk.kind = kind;
    tk.i = i;
    tk.piv = i;
    tk.j = j;
    tk.k = k;
    g.tasks.push_back(tk);
    g.preds.push_back(std::move(pr));
    g.weight.push_back(w);
  };
  // step 1: for each column j, the SYRKs into A(j,j), POTRF(j), the GEMMs
  // below it, the TRSMs (the last writer of each tile also fills L's copy)
  for (int j = 0; j < t; j++) {
    for (int k = 0; k < j; k++) emit(K_CSYRK, j, j, k, {A(j, k)}, {A(j, j)});
    if (inplace)
      emit(K_POTRF, j, j, j, {}, {A(j, j)});
    else
      emit(K_POTRF, j, j, j, {}, {A(j, j), L0(j, j)});
    for (int i = j + 1; i < t; i++)
      for (int k = 0; k < j; k++) emit(K_CGEMM, i, j, k, {A(i, k), A(j, k)}, {A(i, j)});
    for (int i = j + 1; i < t; i++) {
      if (inplace)
        emit(K_CTRSM, i, j, j, {A(j, j)}, {A(i, j)});
      else
        emit(K_CTRSM, i, j, j, {A(j, j)}, {A(i, j), L0(i, j)});
    }
  }
  // step 2: W = L^{-1}, columns from the last; row i of column j is
  // W(i,i) L(i,j), plus W(i,k) L(k,j) over j < k < i, times -W(j,j)
  for (int j = t - 1; j >= 0; j--) {
    if (inplace)
      emit(K_TRTRI, j, j, j, {}, {A(j, j)});
    else
      emit(K_TRTRI, j, j, j, {}, {A(j, j), W0(j, j)});
    for (int i = t - 1; i > j; i--) {
      emit(K_TRMML, i, j, i, {A(i, i)}, {A(i, j)});
      for (int x = 0; x < i - j - 1; x++) {
        const int k = udu ? i - 1 - x : j + 1 + x;
        emit(K_IGEMM, i, j, k, {A(i, k), inplace ? A(k, j) : L0(k, j)}, {A(i, j)});
      }
      if (inplace)
        emit(K_TRMMR, i, j, j, {A(j, j)}, {A(i, j)});
      else
        emit(K_TRMMR, i, j, j, {A(j, j)}, {A(i, j), W0(i, j)});
    }
  }
  // step 3: A^{-1} = W^T W, row block i: W(i,i)^T W(i,j), W(i,i)^T W(i,i),
  // plus W(k,i)^T W(k,j) and W(k,i)^T W(k,i) over k > i
  auto Wsrc = [&](int i, int j) { return inplace ? A(i, j) : W0(i, j); };
  for (int i = 0; i < t; i++) {
    for (int j = 0; j < i; j++) emit(K_TRMMT, i, j, i, {Wsrc(i, i)}, {A(i, j)});
    emit(K_LAUUM, i, i, i, {}, {A(i, i)});
    for (int j = 0; j < i; j++)
      for (int k = i + 1; k < t; k++) emit(K_PGEMM, i, j, k, {Wsrc(k, i), Wsrc(k, j)}, {A(i, j)});
    for (int k = i + 1; k < t; k++) emit(K_PSYRK, i, i, k, {Wsrc(k, i)}, {A(i, i)});
  }
  return g;
}

// ------------------------------------------------- bounded processors
double alap_lost_area(const Graph &g, int P) {
  const int n = (int)g.tasks.size();
  if (n == 0 || P < 1) return 0.0;
  double cp = 0.0;
  for (int t = 0; t < n; t++) cp = std::max(cp, g.bottom[t]);
  // +1 at an ALAP start, -1 at its end; the busy count is constant between
  // consecutive event times.
  std::vector<std::pair<double, int>> ev;
  ev.reserve(2 * (size_t)n);
  for (int t = 0; t < n; t++) {
    const double st = cp - g.bottom[t];
    ev.emplace_back(st, +1);
    ev.emplace_back(st + g.weight[t], -1);
  }
  std::sort(ev.begin(), ev.end());
  // busy[x] holds on [time[x], time[x+1])
  std::vector<double> time;
  std::vector<int> busy;
  int cur = 0;
  for (size_t e = 0; e < ev.size();) {
    const double x = ev[e].first;
    while (e < ev.size() && ev[e].first == x) cur += ev[e++].second;
    time.push_back(x);
    busy.push_back(cur);
  }
  double la = 0.0;
  for (int x = (int)time.size() - 2; x >= 0; x--) {
    if (busy[x] > P) break;
    la += (double)(P - busy[x]) * (time[x + 1] - time[x]);
  }
  return la;
}

double alap_bound(const Graph &g, int P) {
  double cp = 0.0, tseq = 0.0;
  for (size_t t = 0; t < g.tasks.size(); t++) {
    cp = std::max(cp, g.bottom[t]);
    tseq += g.weight[t];
  }
  return std::max(cp, (tseq + alap_lost_area(g, P)) / P);
}

double list_makespan(const Graph &g, int P) {
  const int n = (int)g.tasks.size();
  if (n == 0 || P < 1) return 0.0;
  struct Ready {
    double pri, at;
    int32_t id;
    bool operator<(const Ready &o) const {  // max-heap: the "largest" runs first
      if (pri != o.pri) return pri < o.pri;
      if (at != o.at) return at > o.at;
      return id < o.id;
    }
  };
  std::priority_queue<Ready> ready;
  using Run = std::pair<double, int32_t>;  // (end, id), earliest end first
  std::priority_queue<Run, std::vector<Run>, std::greater<Run>> running;
  std::vector<int32_t> deg(g.indeg0.begin(), g.indeg0.end());
  for (int t = 0; t < n; t++)
    if (deg[t] == 0) ready.push({g.bottom[t], 0.0, t});
  double now = 0.0, makespan = 0.0;
  int idle = P, done = 0;
  while (done < n) {
    while (idle > 0 && !ready.empty()) {
      const Ready r = ready.top();
      ready.pop();
      running.push({now + g.weight[r.id], r.id});
      idle--;
    }
    if (running.empty()) break;  // cannot happen for a valid graph
    now = running.top().first;
    while (!running.empty() && running.top().first == now) {
      const int32_t t = running.top().second;
      running.pop();
      idle++;
      done++;
      makespan = std::max(makespan, now);
      for (int e = g.succ_off[t]; e < g.succ_off[t + 1]; e++) {
        const int32_t s = g.succ[e];
        if (--deg[s] == 0) ready.push({g.bottom[s], now, s});
      }
    }
  }
  return makespan;
}

bool validate(const Graph &g) {
  const int n = (int)g.tasks.size();
  if ((int)g.succ_off.size() != n + 1 || (int)g.indeg0.size() != n) return false;
  std::vector<int32_t> deg(n, 0);
  for (int t = 0; t < n; t++)
    for (int e = g.succ_off[t]; e < g.succ_off[t + 1]; e++) {
      const int32_t s = g.succ[e];
      if (s <= t || s >= n) return false;  // successors come later in list order
      deg[s]++;
    }
  for (int t = 0; t < n; t++)
    if (deg[t] != g.indeg0[t]) return false;
  if (g.static_order) {
    // every task exactly once, each after all its predecessors
    if ((int)g.ready0.size() != n) return false;
    std::vector<int32_t> pos(n, -1);
    for (int x = 0; x < n; x++) {
      const int32_t t = g.ready0[x];
      if (t < 0 || t >= n || pos[t] >= 0) return false;
      pos[t] = x;
    }
    for (int t = 0; t < n; t++)
      for (int e = g.succ_off[t]; e < g.succ_off[t + 1]; e++)
        if (pos[g.succ[e]] <= pos[t]) return false;
    return true;
  }
  std::vector<int32_t> stack(g.ready0.begin(), g.ready0.end());
  int seen = 0;
  while (!stack.empty()) {
    const int32_t t = stack.back();
    stack.pop_back();
    seen++;
    for (int e = g.succ_off[t]; e < g.succ_off[t + 1]; e++)
      if (--deg[g.succ[e]] == 0) stack.push_back(g.succ[e]);
  }
  return seen == n;
}

}  // namespace tqr
