// C ABI of libtqr.so (declared in include/tqr.h): argument checks, the
// per-shape plan cache (task graphs uploaded once per device), workspace
// layout and launches of the device executor.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "graph.h"
#include "mlp.h"
#include "refine.h"
#include "tqr.h"
#include "tqr_types.h"

namespace tqr {
bool zqr_nb_supported(int nb);
int zqr_occupancy(int nb);
hipError_t launch_zqr(const ExecArgs &a, int nb, int grid, int32_t *info, hipStream_t s);
bool cholinv_nb_supported(int nb);
int cholinv_occupancy(int nb);
hipError_t launch_cholinv(const ExecArgs &a, int nb, int grid, int32_t *info, hipStream_t s);
hipError_t launch_exec(const ExecArgs &a, int mode, int grid, const int32_t *order, int32_t *info,
                       hipStream_t s);
int exec_occupancy(int nb, int ib);
bool config_supported(int nb, int ib);
int chunk_width(int nb, int ib);
int config_list(int *nb, int *ib, int cap);
}  // namespace tqr

using namespace tqr;

namespace {

constexpr size_t kHeader = 256;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Plans: factor only; Q^T B only; R X = B only; and the whole least-squares
// solve in one graph (factor, Q^T B and R X = B with the right-hand sides as
// extra tile columns, so B's updates overlap the factorization).
// PK_SNE: R^T Z = B then R X = Z in one graph (semi-normal equations).
enum PlanKind { PK_FACTOR = 0, PK_APPLY = 1, PK_SOLVE = 2, PK_LSTSQ = 3, PK_SOLVET = 4, PK_SNE = 5,
                PK_CHOLINV = 6 /* tile Cholesky inversion: p = q = t, family = renaming, tree = UUU */,
                PK_ZFACTOR = 7, PK_ZAPPLY = 8 /* double complex: the graphs of PK_FACTOR / PK_APPLY */ };
bool solve_kind(int k) { return k == PK_SOLVE || k == PK_SOLVET || k == PK_SNE; }

struct PlanKey {
  int kind, p, q, nbcols, family, tree, param, stripes, stripes_b, priority;
  int nb, P;  // tile size and executor workgroups, for the static order only (else 0)
  bool operator<(const PlanKey &o) const {
    return std::tie(kind, p, q, nbcols, family, tree, param, stripes, stripes_b, priority, nb, P) <
           std::tie(o.kind, o.p, o.q, o.nbcols, o.family, o.tree, o.param, o.stripes, o.stripes_b,
                    o.priority, o.nb, o.P);
  }
};

// Where the static list order pays (measured on MI355X): at nb >= 128
// always (8192^2: 39.6 -> 35.1 ms, 16384 x 2048: 17.3 -> 16.7 ms, batches
// of ragged problems 26.8 -> 22.8 ms); at nb 64 on graphs of up to 64 tasks
// per workgroup (4096 x 1024: 6.4 -> 5.0 ms) but not on larger ones
// (16384 x 2048: 20.1 -> 22.3 ms), whose many short tasks keep workgroups
// busier when taken as they become ready.  Elsewhere the queue is filled
// dynamically in bottom-level order.
bool use_static_order(int nb, size_t ntasks, int P) {
  return nb >= 128 || ntasks <= (size_t)64 * (size_t)std::max(P, 1);
}

struct HostPlan {
  Graph g;
  bool valid = false;
};

struct DevicePlan {
  Task *tasks = nullptr;
  int32_t *succ_off = nullptr, *succ = nullptr, *indeg0 = nullptr, *ready0 = nullptr;
  int32_t ntasks = 0, nready0 = 0;
  int32_t static_order = 0;        // ready0 is a precomputed order of every task
};

// The graph fields of an executor launch, from its device plan.
void set_plan(ExecArgs &a, const DevicePlan &d) {
  a.tasks = d.tasks;
  a.succ_off = d.succ_off;
  a.succ = d.succ;
  a.indeg0 = d.indeg0;
  a.ready0 = d.ready0;
  a.ntasks = d.ntasks;
  a.nready0 = d.nready0;
  a.static_order = d.static_order;
}

std::mutex g_mu;
std::map<PlanKey, std::shared_ptr<HostPlan>> g_host;
std::map<std::pair<int, PlanKey>, DevicePlan> g_dev;
std::map<int, int> g_grid;
std::map<std::pair<int, int>, int64_t> g_spin;
int64_t *g_trace = nullptr;
int64_t g_trace_cap = 0;
// executor launch timing (diagnostics): one event pair per launch
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

std::shared_ptr<HostPlan> host_plan(const PlanKey &k) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_host.find(k);
    if (it != g_host.end()) return it->second;
  }
  auto hp = std::make_shared<HostPlan>();
  if (k.kind == PK_CHOLINV) {
    hp->g = build_cholinv_graph(k.p, k.family == 0, k.tree == 0);
    finalize(hp->g, true);
    if (k.priority == TQR_PRIO_STATIC) static_list_order(hp->g, k.P, k.nb);
    hp->valid = validate(hp->g);
    hp->g.preds.clear();
    hp->g.preds.shrink_to_fit();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_host.find(k);
    if (it != g_host.end()) return it->second;
    g_host[k] = hp;
    return hp;
  }
  GraphSpec spec;
  spec.p = k.p;
  spec.q = k.q;
  spec.family = k.family;
  spec.stripes = k.stripes;
  spec.nbcols = k.nbcols;
  spec.stripes_b = k.stripes_b;
  spec.panels = (k.kind == PK_FACTOR || k.kind == PK_LSTSQ || k.kind == PK_ZFACTOR);
  spec.b_updates = (k.kind == PK_APPLY || k.kind == PK_LSTSQ || k.kind == PK_ZAPPLY);
  spec.solve = (k.kind == PK_SOLVE || k.kind == PK_LSTSQ || k.kind == PK_SNE);
  spec.solve_t = (k.kind == PK_SOLVET || k.kind == PK_SNE);
  std::vector<Elim> list;
  if (!solve_kind(k.kind)) list = make_list(k.tree, k.p, k.q, k.param);
  hp->g = build_graph(list, spec);
  finalize(hp->g, k.priority != 0);
  const bool zkind = (k.kind == PK_ZFACTOR || k.kind == PK_ZAPPLY);
  if (k.priority == TQR_PRIO_STATIC && (zkind || use_static_order(k.nb, hp->g.tasks.size(), k.P)))
    static_list_order(hp->g, k.P, k.nb, zkind);
  hp->valid = validate(hp->g);
  // the host structure is only needed for sequential order and statistics
  hp->g.preds.clear();
  hp->g.preds.shrink_to_fit();
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_host.find(k);
  if (it != g_host.end()) return it->second;
  g_host[k] = hp;
  return hp;
}

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

int device_plan(const PlanKey &k, const HostPlan &hp, int dev, DevicePlan *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, k);
  auto it = g_dev.find(key);
  if (it != g_dev.end()) {
    *out = it->second;
    return TQR_OK;
  }
  DevicePlan d;
  const Graph &g = hp.g;
  if (upload(&d.tasks, g.tasks) != hipSuccess || upload(&d.succ_off, g.succ_off) != hipSuccess ||
      upload(&d.succ, g.succ) != hipSuccess || upload(&d.indeg0, g.indeg0) != hipSuccess ||
      upload(&d.ready0, g.ready0) != hipSuccess)
    return TQR_E_NOMEM;
  d.ntasks = (int32_t)g.tasks.size();
  d.nready0 = (int32_t)g.ready0.size();
  d.static_order = g.static_order ? 1 : 0;
  g_dev[key] = d;
  *out = d;
  return TQR_OK;
}

int grid_size(int dev, int nb, int ib) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_grid.find(dev * 1024 + nb * 4 + ib / 16);
  if (it != g_grid.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 1;
  const int occ = exec_occupancy(nb, ib);
  const int grid = cus * std::max(1, occ);
  g_grid[dev * 1024 + nb * 4 + ib / 16] = grid;
  return grid;
}

// Compute units of the current device (256, MI355X's, when none is visible).
int device_cus() {
  int count = 0, dev = 0, cus = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1 || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 256;
  return cus;
}

// Executor workgroups on the current device, the P of the static list
// order (256, one per CU of MI355X at nb >= 128, when no device is visible).
int current_grid(int nb, int ib) {
  int count = 0, dev = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1 || hipGetDevice(&dev) != hipSuccess) return 256;
  return grid_size(dev, nb, ib);
}

int64_t g_spin_override = 0;  // tqr_debug_spin_limit; 0 = the default below

int64_t spin_limit_ticks(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_spin_override > 0) return g_spin_override;
  auto it = g_spin.find({dev, 0});
  if (it != g_spin.end()) return it->second;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  const int64_t ticks = (int64_t)khz * 1000 * 30;  // 30 s without progress on one slot
  g_spin[{dev, 0}] = ticks;
  return ticks;
}

struct Resolved {
  int nb, ib, tree, param, family, stripes, priority, exec, update_dtype, max_refine, refine_method;
  double refine_tol;
};

// ------------------------------------------------------------- selector
// Registered network (device copy) and its per-shape choices.
struct Selector {
  float *params = nullptr;  // device, kMlpParams floats
  int dev = -1;
  float *scratch = nullptr;  // features and outputs of the candidates
  std::map<std::tuple<int64_t, int64_t, int>, std::array<int, 3>> cache;
};
Selector g_sel;

constexpr int kSelTrees[5] = {TQR_FLAT, TQR_BINARY, TQR_FIBONACCI, TQR_GREEDY, TQR_GRASAP};

int mlp_features(int64_t m, int64_t n, int nb, int tree, int batch, float *out) {
  int slot = -1;
  for (int t = 0; t < 5; t++)
    if (kSelTrees[t] == tree) slot = t;
  if (slot < 0) return -4;
  out[0] = (float)(std::log2((double)m) / 16.0);
  out[1] = (float)(std::log2((double)n) / 16.0);
  out[2] = (float)(std::log2((double)nb) / 8.0);
  for (int t = 0; t < 5; t++) out[3 + t] = (t == slot) ? 1.0f : 0.0f;
  out[8] = (float)(std::log2((double)std::max(batch, 1)) / 10.0);
  return 0;
}

// (tree, nb, ib) of smallest predicted time; GrASAP / 256 / 32 without a
// registered network (or on another device than the one it was registered on).
int select_cfg(int64_t m, int64_t n, int batch, int *tree, int *nb, int *ib) {
  *tree = TQR_GRASAP;
  *nb = 256;
  *ib = 32;
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = -1;
  if (!g_sel.params || hipGetDevice(&dev) != hipSuccess || dev != g_sel.dev) return TQR_OK;
  auto key = std::make_tuple(m, n, batch);
  auto it = g_sel.cache.find(key);
  if (it != g_sel.cache.end()) {
    *tree = it->second[0];
    *nb = it->second[1];
    *ib = it->second[2];
    return TQR_OK;
  }
  int nbs[16], ibs[16];
  const int nc = std::min(config_list(nbs, ibs, 16), 16);
  std::vector<std::array<int, 3>> cand;
  for (int c = 0; c < nc; c++) {
    if (nbs[c] < 64) continue;
    bool better_ib = false;  // one ib per nb: the largest built
    for (int d = 0; d < nc; d++)
      if (nbs[d] == nbs[c] && ibs[d] > ibs[c]) better_ib = true;
    if (better_ib) continue;
    for (int t : kSelTrees) cand.push_back({t, nbs[c], ibs[c]});
  }
  const int K = (int)cand.size();
  std::vector<float> feat((size_t)K * kMlpFeatures), pred((size_t)K);
  for (int k = 0; k < K; k++) mlp_features(m, n, cand[k][1], cand[k][0], batch, &feat[(size_t)k * kMlpFeatures]);
  float *dX = g_sel.scratch, *dY = g_sel.scratch + 1024 * kMlpFeatures;
  if (K > 1024) return TQR_E_INTERNAL;
  if (hipMemcpy(dX, feat.data(), feat.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      mlp_forward(g_sel.params, dX, K, dY, nullptr) != hipSuccess ||
      hipMemcpy(pred.data(), dY, pred.size() * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return TQR_E_HIP;
  int best = 0;
  for (int k = 1; k < K; k++)
    if (pred[k] < pred[best]) best = k;
  *tree = cand[best][0];
  *nb = cand[best][1];
  *ib = cand[best][2];
  g_sel.cache[key] = cand[best];
  return TQR_OK;
}

int resolve(const tqr_opts *o, Resolved *r, int64_t m = 0, int64_t n = 0) {
  tqr_opts d;
  tqr_default_opts(&d);
  const tqr_opts &x = o ? *o : d;
  r->nb = x.nb;
  r->ib = x.ib;
  r->tree = x.tree;
  r->param = x.param;
  r->family = x.kernels;
  r->priority = x.priority;
  r->exec = x.exec;
  if (r->tree == TQR_AUTO) {
    // the learned selector picks tree and tile size for this shape
    int t = TQR_GRASAP, nb = 256, ib = 32;
    if (m > 0 && n > 0) {
      const int rc = select_cfg(m, n, 1, &t, &nb, &ib);
      if (rc) return rc;
    }
    r->tree = t;
    r->param = (t == TQR_GRASAP) ? 1 : 0;
    r->nb = nb;
    r->ib = ib;
  }
  if (!config_supported(r->nb, r->ib)) return TQR_E_UNSUPPORTED;
  if (r->tree < TQR_FLAT || r->tree > TQR_ASAP) return TQR_E_UNSUPPORTED;
  if (r->family != TQR_TT && r->family != TQR_HYBRID) return TQR_E_UNSUPPORTED;
  if (r->exec != TQR_EXEC_PERSISTENT && r->exec != TQR_EXEC_SEQUENTIAL) return TQR_E_UNSUPPORTED;
  if (r->priority < TQR_PRIO_LIST || r->priority > TQR_PRIO_STATIC) return TQR_E_UNSUPPORTED;
  if (x.update_dtype != TQR_F64 && x.update_dtype != TQR_F32 && x.update_dtype != TQR_BF16)
    return TQR_E_UNSUPPORTED;
  r->update_dtype = x.update_dtype;
  r->max_refine = x.max_refine < 0 ? 0 : x.max_refine;
  r->refine_tol = x.refine_tol;
  if (x.refine_method < TQR_REFINE_AUTO || x.refine_method > TQR_REFINE_GMRES) return TQR_E_UNSUPPORTED;
  r->refine_method = x.refine_method;
  const int wc = chunk_width(r->nb, r->ib);
  int s = x.stripes;
  // default: one update task per tile up to nb = 128, four 64-column
  // stripes at nb = 256 (measured: 16384 x 2048 17.2 ms against 17.5 with
  // two stripes and 18.6 with one; at nb 128 one task per tile is fastest)
  if (s <= 0) s = (r->nb >= 256) ? 4 : 1;
  if (s > r->nb / wc) s = r->nb / wc;
  while ((r->nb / wc) % s) s--;  // stripe width is a multiple of the chunk width
  r->stripes = std::max(1, s);
  return TQR_OK;
}

PlanKey make_key(int kind, int p, int q, int64_t nrhs, const Resolved &r) {
  const int nbcols = (kind == PK_FACTOR) ? 0 : (int)cdiv(nrhs, r.nb);
  PlanKey k{};
  k.kind = kind;
  k.p = p;
  k.q = q;
  k.nbcols = nbcols;
  k.family = r.family;
  k.tree = solve_kind(kind) ? 0 : r.tree;
  k.param = solve_kind(kind) ? 0 : r.param;
  k.stripes = r.stripes;
  // right-hand sides narrower than one stripe get one task per tile
  k.stripes_b = (kind == PK_FACTOR || nrhs <= r.nb / r.stripes) ? 1 : r.stripes;
  k.priority = r.priority;
  k.nb = (r.priority == TQR_PRIO_STATIC) ? r.nb : 0;
  k.P = (r.priority == TQR_PRIO_STATIC) ? current_grid(r.nb, r.ib) : 0;
  if (solve_kind(kind)) k.family = 0;
  return k;
}

size_t tfactor_bytes(int64_t p, int64_t q, int nb, int ib) {
  return (size_t)p * q * 2 * ib * nb * sizeof(double);
}

size_t state_bytes(int64_t ntasks) {
  return align_up(sizeof(ExecCtl)) + 2 * align_up((size_t)std::max<int64_t>(ntasks, 1) * 4);
}

// Runs one plan on the device.
int run_plan(int kind, int64_t m, int64_t n, double *A, int64_t lda, double *B, int64_t ldb,
             int64_t nrhs, void *T, size_t t_bytes, const Resolved &r, int32_t *info,
             hipStream_t stream, const int32_t *skip = nullptr, const DevicePlan *given = nullptr) {
  const int nb = r.nb;
  const int64_t p = cdiv(m, nb), q = cdiv(n, nb);
  const PlanKey key = make_key(kind, (int)p, (int)q, kind == PK_FACTOR ? 0 : nrhs, r);
  auto hp = host_plan(key);
  if (!hp->valid) return TQR_E_INTERNAL;
  const size_t tf = tfactor_bytes(p, q, nb, r.ib);
  const size_t need = kHeader + align_up(tf) + state_bytes((int64_t)hp->g.tasks.size());
  if (t_bytes < need) return TQR_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  DevicePlan dp;
  if (given) {
    if (given->ntasks != (int32_t)hp->g.tasks.size()) return TQR_E_INTERNAL;
    dp = *given;
  } else {
    int rc = device_plan(key, *hp, dev, &dp);
    if (rc) return rc;
  }
  char *base = static_cast<char *>(T);
  ExecArgs a{};
  set_plan(a, dp);
  char *st = base + kHeader + align_up(tf);
  a.ctl = reinterpret_cast<ExecCtl *>(st);
  a.queue = reinterpret_cast<int32_t *>(st + align_up(sizeof(ExecCtl)));
  a.indeg = reinterpret_cast<int32_t *>(st + align_up(sizeof(ExecCtl)) +
                                        align_up((size_t)std::max<int32_t>(a.ntasks, 1) * 4));
  a.prob.A = A;
  a.prob.lda = lda;
  a.prob.m = m;
  a.prob.n = n;
  a.prob.B = B;
  a.prob.ldb = ldb;
  a.prob.nrhs = nrhs;
  a.prob.Tf = reinterpret_cast<double *>(base + kHeader);
  a.prob.p = (int)p;
  a.prob.q = (int)q;
  a.prob.sw = nb / key.stripes;
  a.prob.sw_b = nb / key.stripes_b;
  a.prob.dma_ok = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && (lda % 2) == 0) ? 1 : 0;
  a.prob.update_dtype = r.update_dtype;
  a.prob.singular = &a.ctl->pad[0];
  a.prob.skip = nullptr;
  a.probs = nullptr;
  a.nprob = 0;
  a.nb = nb;
  a.ib = r.ib;
  a.skip = skip;
  a.spin_limit = spin_limit_ticks(dev);
  a.trace = g_trace;
  a.trace_cap = g_trace_cap;
  const int grid = grid_size(dev, nb, r.ib);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (g_timing && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess) {
    hipEventRecord(ev0, stream);
  }
  hipError_t e = launch_exec(a, r.exec == TQR_EXEC_SEQUENTIAL ? 1 : 0, grid, hp->g.order.data(),
                             info, stream);
  if (ev1) {
    hipEventRecord(ev1, stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_events.emplace_back(ev0, ev1);
  }
  return e == hipSuccess ? TQR_OK : TQR_E_HIP;
}

int64_t plan_tasks(int kind, int64_t m, int64_t n, int64_t nrhs, const Resolved &r) {
  const int64_t p = cdiv(m, r.nb), q = cdiv(n, r.nb);
  return (int64_t)host_plan(make_key(kind, (int)p, (int)q, kind == PK_FACTOR ? 0 : nrhs, r))->g.tasks.size();
}

// tqr_lstsq's workspace, in order: the refinement report, copies of A and
// B, the factor workspace (T factors and executor state for the largest
// plan), and, with low-precision updates, the refinement buffers: X, the
// residual R (m x nrhs), A^T R (n x nrhs) and the residual partial sums.
struct LsLayout {
  size_t report, ac, bc, t, t_bytes, xw, rw, sw, part, gm, total;
  bool gmres;  // GMRES-based refinement possible (square, one right-hand side)
};

LsLayout ls_layout(int64_t m, int64_t n, int64_t nrhs, const Resolved &r) {
  LsLayout L{};
  int64_t nt = plan_tasks(PK_LSTSQ, m, n, nrhs, r);
  nt = std::max(nt, plan_tasks(PK_FACTOR, m, n, 0, r));
  const bool mixed = r.update_dtype != TQR_F64;
  if (mixed) {
    nt = std::max(nt, plan_tasks(PK_APPLY, m, n, nrhs, r));
    nt = std::max(nt, plan_tasks(PK_SOLVE, m, n, nrhs, r));
    nt = std::max(nt, plan_tasks(PK_SNE, m, n, nrhs, r));
  }
  size_t off = 0;
  L.report = off;
  off += align_up(sizeof(tqr_refine_report));
  L.ac = off;
  off += align_up((size_t)m * n * 8);
  L.bc = off;
  off += align_up((size_t)m * nrhs * 8);
  L.t = off;
  L.t_bytes = kHeader + align_up(tfactor_bytes(cdiv(m, r.nb), cdiv(n, r.nb), r.nb, r.ib)) + state_bytes(nt);
  off += align_up(L.t_bytes);
  if (mixed) {
    L.xw = off;
    off += align_up((size_t)n * nrhs * 8);
    L.rw = off;
    off += align_up((size_t)m * nrhs * 8);
    L.sw = off;
    off += align_up((size_t)n * nrhs * 8);
    L.part = off;
    off += align_up(std::max(refine_partial_bytes(m, n, nrhs),
                             (size_t)kFroBlocks * sizeof(double) + gmres_partial_bytes(n)));
    L.gmres = (m == n && nrhs == 1);
    if (L.gmres) {
      L.gm = off;
      off += align_up(gmres_bytes(n, kGmresMax));
    }
  }
  L.total = off;
  return L;
}


// ------------------------------------------------------------- batches
// A batch of least-squares problems runs as one task graph: the
// concatenation of every problem's graph (tasks carry their problem index),
// with one ready queue ordered by bottom level across problems, in one
// executor launch.  Per-problem data (pointers, sizes, T factors) is in a
// device table indexed by the task's problem.

struct BatchKey {
  int kind, nb, ib, family, stripes, priority;
  int64_t nrhs;
  std::vector<int32_t> shape;  // per problem: p, q, tree, param
  bool operator<(const BatchKey &o) const {
    return std::tie(kind, nb, ib, family, stripes, priority, nrhs, shape) <
           std::tie(o.kind, o.nb, o.ib, o.family, o.stripes, o.priority, o.nrhs, o.shape);
  }
};

struct BatchPlan {
  DevicePlan d;
  std::vector<int32_t> order;  // list order (sequential execution)
  bool valid = false;
};

std::map<std::pair<int, BatchKey>, std::shared_ptr<BatchPlan>> g_batch;

// Tree with the shortest tiled critical path for p x q tiles (the thesis's
// own measure of a tree, section "Critical paths"), among the five trees.
// Kernel family and tree the batch autotuner tries besides (nb, ib): the
// options' own when they name a tree; with TQR_AUTO, the per-problem
// critical-path choice with either family and PlasmaTree domains of 4 and
// 8 tile rows with TS kernels (a batch keeps every CU busy, so kernels that
// do less work per tile can beat shorter critical paths: 512 ragged
// problems at nb 256, 21.8 ms with the per-problem choice and TT kernels,
// 18.9 ms with TS kernels, 17.1 ms with PlasmaTree BS 4 and TS kernels).
struct TreePolicy {
  int family, tree, param;
};
std::vector<TreePolicy> batch_tree_policies(const tqr_opts &o) {
  if (o.tree != TQR_AUTO) return {{o.kernels, o.tree, o.param}};
  return {{TQR_TT, TQR_AUTO, 0}, {TQR_HYBRID, TQR_AUTO, 0}, {TQR_HYBRID, TQR_PLASMA, 4}, {TQR_HYBRID, TQR_PLASMA, 8}};
}

int auto_tree(int p, int q, int family) {
  static std::map<std::tuple<int, int, int>, int> cache;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache.find({p, q, family});
    if (it != cache.end()) return it->second;
  }
  const int cands[] = {TQR_GRASAP, TQR_GREEDY, TQR_FIBONACCI, TQR_BINARY, TQR_FLAT};
  int best = TQR_GRASAP;
  double bcp = 1e300;
  for (int t : cands) {
    GraphSpec spec;
    spec.p = p;
    spec.q = q;
    spec.family = family;
    const Graph g = build_graph(make_list(t, p, q, t == TQR_GRASAP ? 1 : 0), spec);
    if (g.cp < bcp) {
      bcp = g.cp;
      best = t;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  cache[{p, q, family}] = best;
  return best;
}

BatchKey batch_key(int kind, int count, const int64_t *m, const int64_t *n, int64_t nrhs, const Resolved &r,
                   int tree_opt) {
  BatchKey k{};
  k.kind = kind;
  k.nb = r.nb;
  k.ib = r.ib;
  k.family = solve_kind(kind) ? 0 : r.family;
  k.stripes = r.stripes;
  k.priority = r.priority;
  k.nrhs = nrhs;
  k.shape.reserve((size_t)count * 4);
  for (int x = 0; x < count; x++) {
    const int p = (int)cdiv(m[x], r.nb), q = (int)cdiv(n[x], r.nb);
    int tree = tree_opt, param = r.param;
    if (solve_kind(kind)) {
      tree = 0;
      param = 0;
    } else if (tree_opt == TQR_AUTO) {
      tree = auto_tree(p, q, r.family);
      param = (tree == TQR_GRASAP) ? 1 : 0;
    }
    k.shape.insert(k.shape.end(), {p, q, tree, param});
  }
  return k;
}

std::shared_ptr<BatchPlan> batch_plan(const BatchKey &k, const Resolved &r, int dev) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_batch.find({dev, k});
    if (it != g_batch.end()) return it->second;
  }
  auto bp = std::make_shared<BatchPlan>();
  const int count = (int)(k.shape.size() / 4);
  std::vector<Task> tasks;
  std::vector<int32_t> off(1, 0), succ, indeg0;
  std::vector<std::pair<double, int32_t>> ready;
  // with the static order, the list schedule is simulated over the whole
  // concatenated graph (the parts are built with their dynamic ready sets)
  const bool stat = k.priority == TQR_PRIO_STATIC;
  std::vector<double> weight;
  bool valid = true;
  for (int x = 0; x < count; x++) {
    Resolved rx = r;
    rx.priority = std::min(k.priority, (int)TQR_PRIO_BOTTOM);
    rx.tree = k.shape[4 * x + 2];
    rx.param = k.shape[4 * x + 3];
    auto hp = host_plan(make_key(k.kind, k.shape[4 * x], k.shape[4 * x + 1], k.kind == PK_FACTOR ? 0 : k.nrhs, rx));
    valid = valid && hp->valid;
    const Graph &g = hp->g;
    const int32_t base = (int32_t)tasks.size();
    for (size_t t = 0; t < g.tasks.size(); t++) {
      Task tk = g.tasks[t];
      tk.prob = x;
      tasks.push_back(tk);
      for (int32_t e = g.succ_off[t]; e < g.succ_off[t + 1]; e++) succ.push_back(base + g.succ[e]);
      off.push_back((int32_t)succ.size());
      indeg0.push_back(g.indeg0[t]);
      bp->order.push_back(base + (int32_t)t);
      if (stat) weight.push_back(g.weight[t]);
    }
    for (int32_t t : g.ready0) ready.push_back({g.bottom[t], base + t});
  }
  std::stable_sort(ready.begin(), ready.end(),
                   [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
                     return a.first > b.first;
                   });
  std::vector<int32_t> ready0;
  for (auto &pr : ready) ready0.push_back(pr.second);
  bool in_order = false;  // ready0 holds every task in the static order
  if (stat && valid && use_static_order(k.nb, tasks.size(), grid_size(dev, k.nb, k.ib))) {
    in_order = true;
    Graph cg;
    cg.tasks = tasks;
    cg.weight = std::move(weight);
    cg.succ_off = off;
    cg.succ = succ;
    cg.indeg0 = indeg0;
    static_list_order(cg, grid_size(dev, k.nb, k.ib), k.nb);
    valid = validate(cg);
    ready0 = std::move(cg.ready0);
  }
  DevicePlan &d = bp->d;
  if (upload(&d.tasks, tasks) != hipSuccess || upload(&d.succ_off, off) != hipSuccess ||
      upload(&d.succ, succ) != hipSuccess || upload(&d.indeg0, indeg0) != hipSuccess ||
      upload(&d.ready0, ready0) != hipSuccess)
    valid = false;
  d.ntasks = (int32_t)tasks.size();
  d.nready0 = (int32_t)ready0.size();
  d.static_order = in_order ? 1 : 0;
  bp->valid = valid;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_batch.find({dev, k});
  if (it != g_batch.end()) return it->second;
  g_batch[{dev, k}] = bp;
  return bp;
}

// Pinned host staging for the per-call device tables: a ring of buffers per
// device, each reused once the copy that read it last has completed.
struct Staging {
  void *host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
constexpr int kStageRing = 4;
std::map<int, std::pair<int, Staging[kStageRing]>> g_stage;

int stage_copy(int dev, void *dst, const std::vector<char> &src, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto &ring = g_stage[dev];
  Staging &st = ring.second[ring.first];
  ring.first = (ring.first + 1) % kStageRing;
  if (st.done && hipEventSynchronize(st.done) != hipSuccess) return TQR_E_HIP;
  if (st.bytes < src.size()) {
    if (st.host) hipHostFree(st.host);
    st.host = nullptr;
    st.bytes = 0;
    if (hipHostMalloc(&st.host, src.size(), hipHostMallocDefault) != hipSuccess) return TQR_E_NOMEM;
    st.bytes = src.size();
  }
  if (!st.done && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) return TQR_E_HIP;
  std::memcpy(st.host, src.data(), src.size());
  if (hipMemcpyAsync(dst, st.host, src.size(), hipMemcpyHostToDevice, stream) != hipSuccess) return TQR_E_HIP;
  if (hipEventRecord(st.done, stream) != hipSuccess) return TQR_E_HIP;
  return TQR_OK;
}

// Workspace of tqr_lstsq_batched, all offsets 256-byte aligned:
//   reports (count tqr_refine_report, contiguous), device tables (problem
//   tables of the factor and refinement graphs, refinement table, copy
//   descriptors, singular markers), executor state, then per problem: A's
//   copy, B's copy, T factors and, with low-precision updates, the
//   refinement buffers.
struct BatchLayout {
  size_t reports, tables, probs_f, probs_s, refs, copies, sing, state, state_bytes, total;
  std::vector<size_t> ac, bc, tf, xw, rw, sw, part;
  int64_t ntasks_f = 0, ntasks_s = 0;
};

BatchLayout batch_layout(int count, const int64_t *m, const int64_t *n, int64_t nrhs, const Resolved &r,
                         const BatchKey &kf, const BatchKey &ks) {
  BatchLayout L;
  const bool mixed = r.update_dtype != TQR_F64;
  for (int x = 0; x < count; x++) {
    Resolved rx = r;
    rx.tree = kf.shape[4 * x + 2];
    rx.param = kf.shape[4 * x + 3];
    L.ntasks_f += plan_tasks(PK_LSTSQ, m[x], n[x], nrhs, rx);
    if (mixed) L.ntasks_s += plan_tasks(PK_SNE, m[x], n[x], nrhs, rx);
  }
  (void)ks;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.reports = take((size_t)count * sizeof(tqr_refine_report));
  L.tables = off;
  L.probs_f = take((size_t)count * sizeof(Problem));
  L.probs_s = take((size_t)count * sizeof(Problem));
  L.refs = take((size_t)count * sizeof(RefProb));
  L.copies = take((size_t)count * 4 * sizeof(CopyDesc));  // in (A, B), mid, out
  L.sing = take((size_t)count * sizeof(int32_t));
  L.state_bytes = state_bytes(std::max(L.ntasks_f, L.ntasks_s));
  L.state = take(L.state_bytes);
  for (int x = 0; x < count; x++) {
    L.ac.push_back(take((size_t)m[x] * n[x] * 8));
    L.bc.push_back(take((size_t)m[x] * nrhs * 8));
    L.tf.push_back(take(tfactor_bytes(cdiv(m[x], r.nb), cdiv(n[x], r.nb), r.nb, r.ib)));
    if (mixed) {
      L.xw.push_back(take((size_t)n[x] * nrhs * 8));
      L.rw.push_back(take((size_t)m[x] * nrhs * 8));
      L.sw.push_back(take((size_t)n[x] * nrhs * 8));
      L.part.push_back(take(refine_partial_bytes(m[x], n[x], nrhs)));
    }
  }
  L.total = off;
  return L;
}

int check_batch(int count, const int64_t *m, const int64_t *n, int64_t nrhs) {
  if (count < 1) return -1;
  if (!m) return -2;
  if (!n) return -3;
  if (nrhs < 1) return -4;
  for (int x = 0; x < count; x++)
    if (m[x] < 1 || n[x] < 1 || n[x] > m[x]) return -2;
  return TQR_OK;
}

int launch_batch(const BatchPlan &bp, const Resolved &r, int count, ExecCtl *ctl, const Problem *probs,
                 int32_t *info, const int32_t *skip, int dev, hipStream_t stream, size_t state_bytes_) {
  (void)state_bytes_;
  ExecArgs a{};
  set_plan(a, bp.d);
  char *st = reinterpret_cast<char *>(ctl);
  a.ctl = ctl;
  a.queue = reinterpret_cast<int32_t *>(st + align_up(sizeof(ExecCtl)));
  a.indeg = reinterpret_cast<int32_t *>(st + align_up(sizeof(ExecCtl)) +
                                        align_up((size_t)std::max<int32_t>(a.ntasks, 1) * 4));
  a.probs = probs;
  a.nprob = count;
  a.nb = r.nb;
  a.ib = r.ib;
  a.skip = skip;
  a.spin_limit = spin_limit_ticks(dev);
  a.trace = g_trace;
  a.trace_cap = g_trace_cap;
  const int grid = grid_size(dev, r.nb, r.ib);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (g_timing && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess)
    hipEventRecord(ev0, stream);
  hipError_t e = launch_exec(a, r.exec == TQR_EXEC_SEQUENTIAL ? 1 : 0, grid, bp.order.data(), info, stream);
  if (ev1) {
    hipEventRecord(ev1, stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_events.emplace_back(ev0, ev1);
  }
  return e == hipSuccess ? TQR_OK : TQR_E_HIP;
}

}  // namespace

extern "C" {

void tqr_default_opts(tqr_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nb = 256;
  o->ib = 32;
  o->tree = TQR_GREEDY;
  o->kernels = TQR_TT;
  o->param = 0;
  o->update_dtype = TQR_F64;
  o->exec = TQR_EXEC_PERSISTENT;
  o->stripes = 0;
  o->max_refine = 10;
  o->priority = TQR_PRIO_STATIC;
  o->refine_method = TQR_REFINE_AUTO;
  o->refine_tol = 0.0;
}

size_t tqr_workspace_size(int64_t m, int64_t n, int64_t nrhs, const tqr_opts *o) {
  if (m < 1 || n < 1 || n > m || nrhs < 0) return 0;
  Resolved r;
  if (resolve(o, &r, m, n)) return 0;
  const int64_t p = cdiv(m, r.nb), q = cdiv(n, r.nb);
  int64_t nt = plan_tasks(PK_FACTOR, m, n, 0, r);
  if (nrhs > 0) {
    nt = std::max(nt, plan_tasks(PK_APPLY, m, n, nrhs, r));
    nt = std::max(nt, plan_tasks(PK_SOLVE, m, n, nrhs, r));
  }
  return kHeader + align_up(tfactor_bytes(p, q, r.nb, r.ib)) + state_bytes(nt);
}

int tqr_factor_ex(int64_t m, int64_t n, double *A, int64_t lda, void *T, size_t t_bytes,
                  const tqr_opts *o, int32_t *info, hipStream_t stream) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!T) return -5;
  Resolved r;
  int rc = resolve(o, &r, m, n);
  if (rc) return rc;
  return run_plan(PK_FACTOR, m, n, A, lda, nullptr, 0, 0, T, t_bytes, r, info, stream);
}

int tqr_factor(int64_t m, int64_t n, int32_t nb, int32_t tree, double *A, void *T, hipStream_t stream) {
  tqr_opts o;
  tqr_default_opts(&o);
  o.nb = nb;
  o.tree = tree;
  const size_t need = tqr_workspace_size(m, n, 0, &o);
  if (need == 0) return (m < 1) ? -1 : ((n < 1 || n > m) ? -2 : TQR_E_UNSUPPORTED);
  return tqr_factor_ex(m, n, A, m, T, need, &o, nullptr, stream);
}

int tqr_apply_qt(int64_t m, int64_t n, const double *A, int64_t lda, void *T, size_t t_bytes,
                 int64_t nrhs, double *B, int64_t ldb, const tqr_opts *o, int32_t *info,
                 hipStream_t stream) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!T) return -5;
  if (nrhs < 0) return -7;
  if (!B && nrhs > 0) return -8;
  if (ldb < m) return -9;
  if (nrhs == 0) return TQR_OK;
  Resolved r;
  int rc = resolve(o, &r, m, n);
  if (rc) return rc;
  return run_plan(PK_APPLY, m, n, const_cast<double *>(A), lda, B, ldb, nrhs, T, t_bytes, r, info,
                  stream);
}

int tqr_solve_r(int64_t m, int64_t n, const double *A, int64_t lda, void *T, size_t t_bytes,
                int64_t nrhs, double *B, int64_t ldb, const tqr_opts *o, int32_t *info,
                hipStream_t stream) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!T) return -5;
  if (nrhs < 0) return -7;
  if (!B && nrhs > 0) return -8;
  if (ldb < m) return -9;
  if (nrhs == 0) return TQR_OK;
  Resolved r;
  int rc = resolve(o, &r, m, n);
  if (rc) return rc;
  return run_plan(PK_SOLVE, m, n, const_cast<double *>(A), lda, B, ldb, nrhs, T, t_bytes, r, info,
                  stream);
}

size_t tqr_lstsq_work_size(int64_t m, int64_t n, int64_t nrhs, const tqr_opts *o) {
  if (m < 1 || n < 1 || n > m || nrhs < 1) return 0;
  Resolved r;
  if (resolve(o, &r, m, n)) return 0;
  return ls_layout(m, n, nrhs, r).total;
}

}  // extern "C"

namespace {

int lstsq_args(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B, int64_t ldb,
               const double *X, int64_t ldx) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (nrhs < 1) return -3;
  if (!A) return -4;
  if (lda < m) return -5;
  if (!B) return -6;
  if (ldb < m) return -7;
  if (!X) return -8;
  if (ldx < n) return -9;
  return TQR_OK;
}

// The plans one least-squares call runs: the fused solve, and with
// low-precision updates the refinement's Q^T r and R solve (square) or
// semi-normal-equation solve (rectangular).
std::vector<int> lstsq_plan_kinds(int64_t m, int64_t n, const Resolved &r) {
  std::vector<int> k = {PK_LSTSQ};
  if (r.update_dtype != TQR_F64) {
    if (m == n) {
      k.push_back(PK_APPLY);
      k.push_back(PK_SOLVE);
    } else {
      k.push_back(PK_SNE);
    }
  }
  return k;
}

size_t plan_region_bytes(const Graph &g) {
  return align_up(std::max<size_t>(g.tasks.size(), 1) * sizeof(Task)) +
         align_up((g.tasks.size() + 1) * 4) + align_up(std::max<size_t>(g.succ.size(), 1) * 4) +
         2 * align_up(std::max<size_t>(g.tasks.size(), 1) * 4);
}

// Copies a host plan into a device region (stream-ordered) and describes it.
int place_plan(const Graph &g, char *dst, hipStream_t stream, DevicePlan *out) {
  size_t off = 0;
  auto put = [&](auto *&ptr, const auto &vec) -> bool {
    using T = typename std::remove_reference<decltype(vec)>::type::value_type;
    ptr = reinterpret_cast<T *>(dst + off);
    off += align_up(std::max<size_t>(vec.size(), 1) * sizeof(T));
    return vec.empty() || hipMemcpyAsync(ptr, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice,
                                         stream) == hipSuccess;
  };
  Task *t = nullptr;
  int32_t *so = nullptr, *su = nullptr, *i0 = nullptr, *r0 = nullptr;
  if (!put(t, g.tasks) || !put(so, g.succ_off) || !put(su, g.succ) || !put(i0, g.indeg0) || !put(r0, g.ready0))
    return TQR_E_HIP;
  out->tasks = t;
  out->succ_off = so;
  out->succ = su;
  out->indeg0 = i0;
  out->ready0 = r0;
  out->ntasks = (int32_t)g.tasks.size();
  out->nready0 = (int32_t)g.ready0.size();
  out->static_order = g.static_order ? 1 : 0;
  return TQR_OK;
}

// Body of tqr_lstsq.  With plan_area null the task graphs come from the
// library's per-device plan cache; otherwise they are copied into
// plan_area (on the stream) and nothing is allocated on the device.
int lstsq_impl(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B, int64_t ldb,
               double *X, int64_t ldx, void *work, size_t work_bytes, const Resolved &r, int32_t *info,
               hipStream_t stream, char *plan_area) {
  int rc = TQR_OK;
  const LsLayout L = ls_layout(m, n, nrhs, r);
  if (work_bytes < L.total) return TQR_E_WORKSPACE;
  DevicePlan placed[3];
  const DevicePlan *given[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  if (plan_area) {
    const std::vector<int> kinds = lstsq_plan_kinds(m, n, r);
    size_t off = 0;
    for (size_t x = 0; x < kinds.size(); x++) {
      const PlanKey key = make_key(kinds[x], (int)cdiv(m, r.nb), (int)cdiv(n, r.nb), nrhs, r);
      auto hp = host_plan(key);
      if (!hp->valid) return TQR_E_INTERNAL;
      rc = place_plan(hp->g, plan_area + off, stream, &placed[x]);
      if (rc) return rc;
      off += plan_region_bytes(hp->g);
      given[kinds[x]] = &placed[x];
    }
  }
  char *w = static_cast<char *>(work);
  double *Ac = reinterpret_cast<double *>(w + L.ac);
  double *Bc = reinterpret_cast<double *>(w + L.bc);
  char *T = w + L.t;
  auto *rep = reinterpret_cast<RefineState *>(w + L.report);
  if (hipMemcpy2DAsync(Ac, m * 8, A, lda * 8, m * 8, n, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return TQR_E_HIP;
  if (hipMemcpy2DAsync(Bc, m * 8, B, ldb * 8, m * 8, nrhs, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return TQR_E_HIP;
  {
    RefProb P0{};
    P0.st = rep;
    if (refine_start(nullptr, P0, 1, stream) != hipSuccess) return TQR_E_HIP;
  }
  // factorization, Q^T B and R X = (Q^T B)(1:n) in one executor launch
  rc = run_plan(PK_LSTSQ, m, n, Ac, m, Bc, m, nrhs, T, L.t_bytes, r, info, stream, nullptr, given[PK_LSTSQ]);
  if (rc) return rc;
  if (r.update_dtype == TQR_F64) {
    if (hipMemcpy2DAsync(X, ldx * 8, Bc, m * 8, n * 8, nrhs, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return TQR_E_HIP;
    return TQR_OK;
  }
  // Low-precision updates: refine X in FP64 against the caller's A and B.
  // Square systems use classical refinement, d = R^{-1} (Q^T r)(1:n), or
  // GMRES on A d = r preconditioned by M^{-1} = R^{-1} Q^T; rectangular
  // ones the semi-normal equations with the computed R, d = R^{-1} R^{-T}
  // A^T r, whose fixed point satisfies A^T r = 0 exactly (classical
  // refinement would stop at a point with A^T r of the size of the
  // factorization error times r).  Unless the stream is being captured,
  // the report is read back after each test: no step is enqueued after
  // convergence, a classical step that fails to halve the backward error
  // switches a square one-right-hand-side system to GMRES (method AUTO),
  // and a GMRES step that fails to halve it ends the refinement.  Under
  // capture every step is enqueued and the kernels of the steps after
  // convergence return at once.
  const bool square = (m == n);
  RefProb P{};
  P.A = A;
  P.lda = lda;
  P.m = m;
  P.n = n;
  P.B = B;
  P.ldb = ldb;
  P.nrhs = nrhs;
  P.X = reinterpret_cast<double *>(w + L.xw);
  P.ldx = n;
  P.R = reinterpret_cast<double *>(w + L.rw);
  P.ldr = m;
  P.S = square ? nullptr : reinterpret_cast<double *>(w + L.sw);
  P.lds = n;
  P.partial = w + L.part;
  P.st = rep;
  P.info = info;
  P.square = square ? 1 : 0;
  const double tol = r.refine_tol > 0.0 ? r.refine_tol : 16.0 * 2.220446049250313e-16;
  const int32_t *skip = &rep->done;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  const bool poll = hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone;
  const bool can_gmres = poll && L.gmres && r.refine_method != TQR_REFINE_CLASSICAL;
  bool use_gmres = can_gmres && r.refine_method == TQR_REFINE_GMRES;
  bool last_gmres = false;  // the previous step was a GMRES step
  GmArgs G{};
  if (can_gmres)
    G = gmres_args(w + L.gm, n, kGmresMax, A, lda, P.X, P.R, w + L.part + kFroBlocks * sizeof(double), rep,
                   1e-4);
  // M^{-1} z = R^{-1} (Q^T z)(1:n) in place on the m x nrhs buffer z
  auto precondition = [&](double *z) -> int {
    int e = run_plan(PK_APPLY, m, n, Ac, m, z, m, nrhs, T, L.t_bytes, r, info, stream, skip, given[PK_APPLY]);
    if (!e) e = run_plan(PK_SOLVE, m, n, Ac, m, z, m, nrhs, T, L.t_bytes, r, info, stream, skip, given[PK_SOLVE]);
    return e;
  };
  tqr_refine_report host{};
  auto read_back = [&](void *dst, const void *src, size_t bytes) -> bool {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream) == hipSuccess &&
           hipStreamSynchronize(stream) == hipSuccess;
  };
  if (hipMemcpy2DAsync(P.X, n * 8, Bc, m * 8, n * 8, nrhs, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return TQR_E_HIP;
  if (refine_fro(nullptr, P, 1, stream) != hipSuccess) return TQR_E_HIP;
  for (int it = 0; it <= r.max_refine; it++) {
    if (refine_residual(nullptr, P, 1, m, n, stream) != hipSuccess) return TQR_E_HIP;
    if (refine_check(nullptr, P, 1, tol, it, stream) != hipSuccess) return TQR_E_HIP;
    if (it == r.max_refine) break;
    if (poll) {
      if (!read_back(&host, rep, sizeof(host))) return TQR_E_HIP;
      if (host.done) break;
      const bool stalled = it >= 1 && it < kRefineHistory && !(host.history[it] <= 0.5 * host.history[it - 1]);
      // a GMRES step that fails to halve the error: the factors are too far
      // from A for this method; stop (info reports NOCONV) rather than
      // spend the remaining steps
      if (stalled && use_gmres && last_gmres) break;
      if (stalled && can_gmres) use_gmres = true;
    }
    last_gmres = use_gmres;
    if (use_gmres) {
      // one GMRES cycle on A d = r: z = M^{-1} r, then Krylov steps with
      // z = M^{-1} A v_j until the preconditioned residual has dropped by
      // the cycle's tolerance; x += V y
      rc = precondition(P.R);
      if (rc) return rc;
      if (gmres_init(G, stream) != hipSuccess) return TQR_E_HIP;
      for (int j = 0; j < kGmresMax; j++) {
        if (gmres_matvec(G, j, stream) != hipSuccess) return TQR_E_HIP;
        rc = precondition(P.R);
        if (rc) return rc;
        if (gmres_arnoldi(G, j, stream) != hipSuccess) return TQR_E_HIP;
        GmState gs{};
        if (!read_back(&gs, G.st, sizeof(gs))) return TQR_E_HIP;
        if (gs.inner_done) break;
      }
      if (gmres_update(G, stream) != hipSuccess) return TQR_E_HIP;
      continue;
    }
    if (square) {
      rc = precondition(P.R);
    } else {
      rc = run_plan(PK_SNE, m, n, Ac, m, P.S, n, nrhs, T, L.t_bytes, r, info, stream, skip, given[PK_SNE]);
    }
    if (rc) return rc;
    if (refine_update(nullptr, P, 1, n, nrhs, stream) != hipSuccess) return TQR_E_HIP;
  }
  if (refine_finish(nullptr, P, 1, TQR_INFO_NOCONV, stream) != hipSuccess) return TQR_E_HIP;
  double *xw = P.X;
  if (hipMemcpy2DAsync(X, ldx * 8, xw, n * 8, n * 8, nrhs, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return TQR_E_HIP;
  return TQR_OK;
}

}  // namespace

namespace tqr {

// The allocation-free least-squares solve (called by tqr_lstsq_noalloc with
// its device's scratch array): the workspace and the task graphs share
// `scratch`; TQR_E_SCRATCH when they do not fit.
int lstsq_scratch(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                  int64_t ldb, double *X, int64_t ldx, const tqr_opts *o, int32_t *info, hipStream_t stream,
                  char *scratch, size_t scratch_bytes) {
  int rc = lstsq_args(m, n, nrhs, A, lda, B, ldb, X, ldx);
  if (rc) return rc;
  if (o && o->tree == TQR_AUTO) return TQR_E_UNSUPPORTED;  // the selector runs device work
  Resolved r;
  rc = resolve(o, &r, m, n);
  if (rc) return rc;
  const LsLayout L = ls_layout(m, n, nrhs, r);
  size_t plans = 0;
  for (int kind : lstsq_plan_kinds(m, n, r))
    plans += plan_region_bytes(host_plan(make_key(kind, (int)cdiv(m, r.nb), (int)cdiv(n, r.nb), nrhs, r))->g);
  const size_t work = align_up(L.total);
  if (work + plans > scratch_bytes) return TQR_E_SCRATCH;
  return lstsq_impl(m, n, nrhs, A, lda, B, ldb, X, ldx, scratch, work, r, info, stream, scratch + work);
}

}  // namespace tqr

extern "C" {

int tqr_lstsq(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
              int64_t ldb, double *X, int64_t ldx, void *work, size_t work_bytes, const tqr_opts *o,
              int32_t *info, hipStream_t stream) {
  int rc = lstsq_args(m, n, nrhs, A, lda, B, ldb, X, ldx);
  if (rc) return rc;
  if (!work) return -10;
  Resolved r;
  rc = resolve(o, &r, m, n);
  if (rc) return rc;
  return lstsq_impl(m, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes, r, info, stream, nullptr);
}

size_t tqr_lstsq_batched_work_size(int32_t count, const int64_t *m, const int64_t *n, int64_t nrhs,
                                   const tqr_opts *o) {
  if (check_batch(count, m, n, nrhs)) return 0;
  tqr_opts d;
  tqr_default_opts(&d);
  const tqr_opts x0 = o ? *o : d;
  int nbs[16], ibs[16];
  int nc = 1;
  if (x0.nb == 0) {
    nc = std::min(config_list(nbs, ibs, 16), 16);
  } else {
    nbs[0] = x0.nb;
    ibs[0] = x0.ib;
  }
  size_t best = 0;
  // with nb == 0 (the autotuner's workspace): also over its tree policies
  const std::vector<TreePolicy> pol = x0.nb == 0 ? batch_tree_policies(x0)
                                                 : std::vector<TreePolicy>{{x0.kernels, x0.tree, x0.param}};
  for (const TreePolicy &tp : pol)
    for (int c = 0; c < nc; c++) {
      tqr_opts x = x0;
      x.nb = nbs[c];
      x.ib = ibs[c];
      x.kernels = tp.family;
      x.param = tp.param;
      const int tree_opt = tp.tree;
      x.tree = tp.tree == TQR_AUTO ? TQR_GRASAP : tp.tree;  // per-problem choice below; nb from opts
      Resolved r;
      if (resolve(&x, &r)) return 0;
      const BatchKey kf = batch_key(PK_LSTSQ, count, m, n, nrhs, r, tree_opt);
      const BatchKey ks = batch_key(PK_SNE, count, m, n, nrhs, r, tree_opt);
      best = std::max(best, batch_layout(count, m, n, nrhs, r, kf, ks).total);
    }
  return best;
}

int tqr_lstsq_batched(int32_t count, const int64_t *m, const int64_t *n, int64_t nrhs, const double *const *A,
                      const int64_t *lda, const double *const *B, const int64_t *ldb, double *const *X,
                      const int64_t *ldx, void *work, size_t work_bytes, const tqr_opts *o, int32_t *info,
                      hipStream_t stream) {
  int rc = check_batch(count, m, n, nrhs);
  if (rc) return rc;
  if (!A || !lda || !B || !ldb || !X || !ldx) return -5;
  for (int x = 0; x < count; x++) {
    if (!A[x] || lda[x] < m[x]) return -5;
    if (!B[x] || ldb[x] < m[x]) return -7;
    if (!X[x] || ldx[x] < n[x]) return -9;
  }
  if (!work) return -11;
  tqr_opts d;
  tqr_default_opts(&d);
  tqr_opts oc = o ? *o : d;
  const int tree_opt = oc.tree;
  if (oc.tree == TQR_AUTO) oc.tree = TQR_GRASAP;  // per-problem choice in batch_key; nb from opts
  Resolved r;
  rc = resolve(&oc, &r);
  if (rc) return rc;
  const bool mixed = r.update_dtype != TQR_F64;
  const BatchKey kf = batch_key(PK_LSTSQ, count, m, n, nrhs, r, tree_opt);
  const BatchKey ks = batch_key(PK_SNE, count, m, n, nrhs, r, tree_opt);
  const BatchLayout L = batch_layout(count, m, n, nrhs, r, kf, ks);
  if (work_bytes < L.total) return TQR_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  auto bpf = batch_plan(kf, r, dev);
  if (!bpf->valid) return TQR_E_INTERNAL;
  std::shared_ptr<BatchPlan> bps;
  if (mixed) {
    bps = batch_plan(ks, r, dev);
    if (!bps->valid) return TQR_E_INTERNAL;
  }
  char *w = static_cast<char *>(work);
  auto *reports = reinterpret_cast<RefineState *>(w + L.reports);
  auto *sing = reinterpret_cast<int32_t *>(w + L.sing);
  // device tables, staged in one copy
  std::vector<char> tab(L.state - L.tables, 0);
  auto at = [&](size_t off) { return tab.data() + (off - L.tables); };
  auto *pf = reinterpret_cast<Problem *>(at(L.probs_f));
  auto *ps = reinterpret_cast<Problem *>(at(L.probs_s));
  auto *rf = reinterpret_cast<RefProb *>(at(L.refs));
  auto *cp = reinterpret_cast<CopyDesc *>(at(L.copies));
  int64_t mmax = 0, nmax = 0, emax = 0;
  for (int x = 0; x < count; x++) {
    double *Ac = reinterpret_cast<double *>(w + L.ac[x]);
    double *Bc = reinterpret_cast<double *>(w + L.bc[x]);
    const int stripes_b = (nrhs <= r.nb / r.stripes) ? 1 : r.stripes;
    Problem P{};
    P.A = Ac;
    P.lda = m[x];
    P.m = m[x];
    P.n = n[x];
    P.B = Bc;
    P.ldb = m[x];
    P.nrhs = nrhs;
    P.Tf = reinterpret_cast<double *>(w + L.tf[x]);
    P.p = (int)cdiv(m[x], r.nb);
    P.q = (int)cdiv(n[x], r.nb);
    P.sw = r.nb / r.stripes;
    P.sw_b = r.nb / stripes_b;
    P.dma_ok = (m[x] % 2 == 0) ? 1 : 0;
    P.update_dtype = r.update_dtype;
    P.singular = sing + x;
    P.skip = nullptr;
    pf[x] = P;
    cp[2 * x] = CopyDesc{A[x], lda[x], Ac, m[x], m[x], n[x]};
    cp[2 * x + 1] = CopyDesc{B[x], ldb[x], Bc, m[x], m[x], nrhs};
    mmax = std::max(mmax, m[x]);
    nmax = std::max(nmax, n[x]);
    emax = std::max(emax, m[x] * std::max(n[x], nrhs));
    RefProb R{};
    R.st = reports + x;
    R.info = info ? info + x : nullptr;
    if (mixed) {
      double *sw = reinterpret_cast<double *>(w + L.sw[x]);
      Problem Q = P;
      Q.B = sw;
      Q.ldb = n[x];
      Q.skip = &reports[x].done;
      ps[x] = Q;
      R.A = A[x];
      R.lda = lda[x];
      R.m = m[x];
      R.n = n[x];
      R.B = B[x];
      R.ldb = ldb[x];
      R.nrhs = nrhs;
      R.X = reinterpret_cast<double *>(w + L.xw[x]);
      R.ldx = n[x];
      R.R = reinterpret_cast<double *>(w + L.rw[x]);
      R.ldr = m[x];
      R.S = sw;
      R.lds = n[x];
      R.partial = w + L.part[x];
      // the correction always comes from the semi-normal equations (S);
      // the stopping test of a square member is Rigal-Gaches, whose
      // residual reaches rounding level (Stewart's bound would stay near
      // 1/kappa for a consistent system)
      R.square = (m[x] == n[x]) ? 1 : 0;
    }
    rf[x] = R;
  }
  // result copies: X = first n rows of the solved B copies (of the refined
  // iterate with low-precision updates); with refinement the iterate starts
  // from the solved B copies
  for (int x = 0; x < count; x++) {
    double *bc = reinterpret_cast<double *>(w + L.bc[x]);
    if (mixed) {
      double *xw = reinterpret_cast<double *>(w + L.xw[x]);
      cp[2 * count + x] = CopyDesc{bc, m[x], xw, n[x], n[x], nrhs};
      cp[3 * count + x] = CopyDesc{xw, n[x], X[x], ldx[x], n[x], nrhs};
    } else {
      cp[3 * count + x] = CopyDesc{bc, m[x], X[x], ldx[x], n[x], nrhs};
    }
  }
  rc = stage_copy(dev, w + L.tables, tab, stream);
  if (rc) return rc;
  const RefProb none{};
  const auto *dref = reinterpret_cast<const RefProb *>(w + L.refs);
  const auto *dcp = reinterpret_cast<const CopyDesc *>(w + L.copies);
  if (copy_batch(dcp, 2 * count, emax, stream) != hipSuccess) return TQR_E_HIP;
  if (refine_start(dref, none, count, stream) != hipSuccess) return TQR_E_HIP;
  auto *ctl = reinterpret_cast<ExecCtl *>(w + L.state);
  rc = launch_batch(*bpf, r, count, ctl, reinterpret_cast<const Problem *>(w + L.probs_f), info, nullptr, dev,
                    stream, L.state_bytes);
  if (rc) return rc;
  if (mixed) {
    if (copy_batch(dcp + 2 * count, count, nmax * nrhs, stream) != hipSuccess) return TQR_E_HIP;
    const double tol = r.refine_tol > 0.0 ? r.refine_tol : 16.0 * 2.220446049250313e-16;
    if (refine_fro(dref, none, count, stream) != hipSuccess) return TQR_E_HIP;
    // Unless the stream is being captured, the reports are read back after
    // each test and no step is enqueued once every problem has converged
    // (under capture every step is enqueued; converged problems' kernels
    // return at once).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool poll = hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone;
    std::vector<tqr_refine_report> host(poll ? count : 0);
    for (int it = 0; it <= r.max_refine; it++) {
      if (refine_residual(dref, none, count, mmax, nmax, stream) != hipSuccess) return TQR_E_HIP;
      if (refine_check(dref, none, count, tol, it, stream) != hipSuccess) return TQR_E_HIP;
      if (it == r.max_refine) break;
      if (poll) {
        if (hipMemcpyAsync(host.data(), reports, (size_t)count * sizeof(tqr_refine_report), hipMemcpyDeviceToHost,
                           stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
          return TQR_E_HIP;
        bool all = true;
        for (int x = 0; x < count && all; x++) all = host[x].done != 0;
        if (all) break;
      }
      rc = launch_batch(*bps, r, count, ctl, reinterpret_cast<const Problem *>(w + L.probs_s), info, nullptr,
                        dev, stream, L.state_bytes);
      if (rc) return rc;
      if (refine_update(dref, none, count, nmax, nrhs, stream) != hipSuccess) return TQR_E_HIP;
    }
    if (refine_finish(dref, none, count, TQR_INFO_NOCONV, stream) != hipSuccess) return TQR_E_HIP;
  }
  if (copy_batch(dcp + 3 * count, count, nmax * nrhs, stream) != hipSuccess) return TQR_E_HIP;
  return TQR_OK;
}

int tqr_autotune_batched(int32_t count, const int64_t *m, const int64_t *n, int64_t nrhs, const double *const *A,
                         const int64_t *lda, const double *const *B, const int64_t *ldb, double *const *X,
                         const int64_t *ldx, void *work, size_t work_bytes, tqr_opts *o, float *best_ms,
                         hipStream_t stream) {
  if (!o) return -13;
  int rc = check_batch(count, m, n, nrhs);
  if (rc) return rc;
  // the choice (nb, ib, kernels, tree, param), cached under the options
  // given and under the options chosen
  static std::map<std::vector<int64_t>, std::array<int, 5>> cache;
  auto signature = [&](const tqr_opts &q) {
    std::vector<int64_t> sig = {count, nrhs, q.tree, q.kernels, q.update_dtype, q.param, q.stripes};
    for (int x = 0; x < count; x++) {
      sig.push_back(m[x]);
      sig.push_back(n[x]);
    }
    return sig;
  };
  const std::vector<int64_t> sig = signature(*o);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache.find(sig);
    if (it != cache.end()) {
      o->nb = it->second[0];
      o->ib = it->second[1];
      o->kernels = it->second[2];
      o->tree = it->second[3];
      o->param = it->second[4];
      if (best_ms) *best_ms = -1.0f;
      return TQR_OK;
    }
  }
  int nbs[16], ibs[16];
  const int nc = std::min(config_list(nbs, ibs, 16), 16);
  const std::vector<TreePolicy> pol = batch_tree_policies(*o);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TQR_E_HIP;
  float bms = 1e30f;
  int bnb = 0, bib = 0;
  TreePolicy bpol = pol[0];
  for (int c = 0; c < nc * (int)pol.size(); c++) {
    tqr_opts x = *o;
    x.nb = nbs[c % nc];
    x.ib = ibs[c % nc];
    const TreePolicy &tp = pol[c / nc];
    x.kernels = tp.family;
    x.tree = tp.tree;
    x.param = tp.param;
    // first run builds and uploads the plans; the second is timed
    rc = tqr_lstsq_batched(count, m, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes, &x, nullptr, stream);
    if (rc == TQR_E_WORKSPACE) continue;
    if (rc) break;
    hipEventRecord(e0, stream);
    rc = tqr_lstsq_batched(count, m, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes, &x, nullptr, stream);
    hipEventRecord(e1, stream);
    if (rc) break;
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = TQR_E_HIP;
      break;
    }
    if (ms < bms) {
      bms = ms;
      bnb = x.nb;
      bib = x.ib;
      bpol = tp;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (bnb == 0) return TQR_E_WORKSPACE;
  o->nb = bnb;
  o->ib = bib;
  o->kernels = bpol.family;
  o->tree = bpol.tree;
  o->param = bpol.param;
  if (best_ms) *best_ms = bms;
  const std::array<int, 5> choice = {bnb, bib, bpol.family, bpol.tree, bpol.param};
  std::lock_guard<std::mutex> lk(g_mu);
  cache[sig] = choice;
  cache[signature(*o)] = choice;
  return TQR_OK;
}

int32_t tqr_mlp_params(void) { return kMlpParams; }
int32_t tqr_mlp_features(void) { return kMlpFeatures; }

int tqr_mlp_features_of(int64_t m, int64_t n, int32_t nb, int32_t tree, int32_t batch, float *out) {
  if (m < 1 || n < 1) return -1;
  if (nb < 1) return -3;
  if (!out) return -6;
  return mlp_features(m, n, nb, tree, batch, out);
}

size_t tqr_mlp_work_size(int64_t batch) { return batch < 1 ? 0 : mlp_work_bytes(batch); }

int tqr_mlp_forward(const float *params, const float *X, int64_t batch, float *y, hipStream_t stream) {
  if (!params) return -1;
  if (!X) return -2;
  if (batch < 1) return -3;
  if (!y) return -4;
  return mlp_forward(params, X, batch, y, stream) == hipSuccess ? TQR_OK : TQR_E_HIP;
}

int tqr_mlp_grad(const float *params, const float *X, const float *target, int64_t batch, float *grad,
                 float *loss, void *work, size_t work_bytes, hipStream_t stream) {
  if (!params) return -1;
  if (!X) return -2;
  if (!target) return -3;
  if (batch < 1) return -4;
  if (!grad) return -5;
  if (!work) return -7;
  if (work_bytes < mlp_work_bytes(batch)) return TQR_E_WORKSPACE;
  return mlp_grad(params, X, target, batch, grad, loss, work, stream) == hipSuccess ? TQR_OK : TQR_E_HIP;
}

int tqr_mlp_adam(float *params, const float *grad, float *m1, float *m2, int64_t step, float lr,
                 hipStream_t stream) {
  if (!params) return -1;
  if (!grad) return -2;
  if (!m1) return -3;
  if (!m2) return -4;
  if (step < 1) return -5;
  return mlp_adam(params, grad, m1, m2, step, lr, stream) == hipSuccess ? TQR_OK : TQR_E_HIP;
}

int tqr_mlp_fit(float *params, const float *X, const float *target, int64_t batch, int32_t epochs, float lr,
                float *loss_hist, void *work, size_t work_bytes, hipStream_t stream) {
  if (!params) return -1;
  if (!X) return -2;
  if (!target) return -3;
  if (batch < 1) return -4;
  if (epochs < 0) return -5;
  if (!work) return -8;
  if (work_bytes < mlp_work_bytes(batch)) return TQR_E_WORKSPACE;
  // work: per-sample gradients and errors (used by mlp_grad), then the
  // summed gradient and Adam's two moment vectors
  float *grad = static_cast<float *>(work) + (size_t)batch * kMlpParams + (size_t)batch;
  float *m1 = grad + kMlpParams;
  float *m2 = m1 + kMlpParams;
  if (mlp_zero(m1, 2 * (int64_t)kMlpParams, stream) != hipSuccess) return TQR_E_HIP;
  for (int32_t e = 0; e < epochs; e++) {
    if (mlp_grad(params, X, target, batch, grad, loss_hist ? loss_hist + e : nullptr, work, stream) != hipSuccess)
      return TQR_E_HIP;
    if (mlp_adam(params, grad, m1, m2, e + 1, lr, stream) != hipSuccess) return TQR_E_HIP;
  }
  return TQR_OK;
}

int tqr_set_selector(const float *params) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_sel.cache.clear();
  if (!params) {
    if (g_sel.params) hipFree(g_sel.params);
    if (g_sel.scratch) hipFree(g_sel.scratch);
    g_sel.params = nullptr;
    g_sel.scratch = nullptr;
    g_sel.dev = -1;
    return TQR_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  if (!g_sel.params && hipMalloc(&g_sel.params, kMlpParams * sizeof(float)) != hipSuccess) return TQR_E_NOMEM;
  if (!g_sel.scratch && hipMalloc(&g_sel.scratch, 1024 * (kMlpFeatures + 1) * sizeof(float)) != hipSuccess)
    return TQR_E_NOMEM;
  if (hipMemcpy(g_sel.params, params, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice) != hipSuccess)
    return TQR_E_HIP;
  g_sel.dev = dev;
  return TQR_OK;
}

int tqr_select(int64_t m, int64_t n, int32_t batch, int32_t *tree, int32_t *nb, int32_t *ib) {
  if (m < 1 || n < 1 || n > m) return -1;
  int t, b, i;
  const int rc = select_cfg(m, n, batch, &t, &b, &i);
  if (rc) return rc;
  if (tree) *tree = t;
  if (nb) *nb = b;
  if (ib) *ib = i;
  return TQR_OK;
}

int64_t tqr_tree_list(int32_t tree, int32_t p, int32_t q, int32_t param, int32_t *i_out,
                      int32_t *piv_out, int32_t *k_out, int64_t cap) {
  if (p < 1 || q < 1 || q > p) return -2;
  if (tree < TQR_FLAT || tree > TQR_ASAP) return -1;
  std::vector<Elim> l = make_list(tree, p, q, param);
  if ((int64_t)l.size() <= cap && i_out && piv_out && k_out)
    for (size_t e = 0; e < l.size(); e++) {
      i_out[e] = l[e].i + 1;
      piv_out[e] = l[e].piv + 1;
      k_out[e] = l[e].k + 1;
    }
  return (int64_t)l.size();
}

int64_t tqr_tree_cp(int32_t tree, int32_t p, int32_t q, int32_t param, int32_t kernels,
                    int64_t *zero_t, int64_t *counts) {
  if (p < 1 || q < 1 || q > p) return -2;
  if (tree < TQR_FLAT || tree > TQR_ASAP) return -1;
  if (kernels != TQR_TT && kernels != TQR_HYBRID) return -5;
  std::vector<Elim> l = make_list(tree, p, q, param);
  GraphSpec spec;
  spec.p = p;
  spec.q = q;
  spec.family = kernels;
  std::vector<double> zt;
  Graph g = build_graph(l, spec, &zt, nullptr);
  if (zero_t)
    for (size_t x = 0; x < zt.size(); x++) zero_t[x] = (int64_t)zt[x];
  if (counts) {
    for (int c = 0; c < 6; c++) counts[c] = 0;
    for (const Task &t : g.tasks)
      if (t.kind < 6) counts[t.kind]++;
  }
  return (int64_t)g.cp;
}

int tqr_graph_stats(int64_t m, int64_t n, const tqr_opts *o, int64_t *ntasks, int64_t *nedges) {
  if (m < 1 || n < 1 || n > m) return -1;
  Resolved r;
  int rc = resolve(o, &r, m, n);
  if (rc) return rc;
  auto hp = host_plan(make_key(PK_FACTOR, (int)cdiv(m, r.nb), (int)cdiv(n, r.nb), 0, r));
  if (ntasks) *ntasks = (int64_t)hp->g.tasks.size();
  if (nedges) *nedges = hp->g.nedges;
  return hp->valid ? TQR_OK : TQR_E_INTERNAL;
}

// ------------------------------------------------ double-complex tiled QR
}  // extern "C"

namespace {

struct ZResolved {
  int nb, tree, param, family;
};

int zresolve(const tqr_opts *o, ZResolved *z) {
  tqr_opts d;
  tqr_default_opts(&d);
  const tqr_opts &x = o ? *o : d;
  z->nb = o ? x.nb : 64;
  z->tree = x.tree;
  z->param = x.param;
  z->family = x.kernels;
  if (!zqr_nb_supported(z->nb)) return TQR_E_UNSUPPORTED;
  if (z->tree < TQR_FLAT || z->tree > TQR_ASAP) return TQR_E_UNSUPPORTED;
  if (z->family != TQR_TT && z->family != TQR_HYBRID) return TQR_E_UNSUPPORTED;
  if (z->tree == TQR_GRASAP && z->param < 1) z->param = 1;
  return TQR_OK;
}

PlanKey zkey(int kind, int64_t m, int64_t n, int64_t nrhs, const ZResolved &z) {
  PlanKey k{};
  k.kind = kind;
  k.p = (int)cdiv(m, z.nb);
  k.q = (int)cdiv(n, z.nb);
  k.nbcols = (kind == PK_ZFACTOR) ? 0 : (int)cdiv(nrhs, z.nb);
  k.family = z.family;
  k.tree = z.tree;
  k.param = z.param;
  k.stripes = k.stripes_b = 1;
  // nb 64: the static list order with the complex kernels' measured costs;
  // nb 32 (no cost measurements): the dynamic queue
  if (z.nb == 64) {
    k.priority = TQR_PRIO_STATIC;
    k.nb = z.nb;
    k.P = device_cus() * zqr_occupancy(z.nb);
  } else {
    k.priority = TQR_PRIO_BOTTOM;
  }
  return k;
}

size_t ztau_bytes(int64_t m, int64_t n, int nb) { return (size_t)cdiv(m, nb) * cdiv(n, nb) * 2 * nb * 16; }

size_t zwork_bytes(int64_t m, int64_t n, int64_t nrhs, const ZResolved &z) {
  int64_t nt = (int64_t)host_plan(zkey(PK_ZFACTOR, m, n, 0, z))->g.tasks.size();
  if (nrhs > 0) nt = std::max(nt, (int64_t)host_plan(zkey(PK_ZAPPLY, m, n, nrhs, z))->g.tasks.size());
  return align_up(ztau_bytes(m, n, z.nb)) + state_bytes(nt);
}

std::map<std::pair<int, int>, int> g_z_grid;

int zrun(int kind, int64_t m, int64_t n, void *A, int64_t lda, void *B, int64_t ldb, int64_t nrhs, void *W,
         size_t w_bytes, const ZResolved &z, int32_t *info, hipStream_t stream) {
  const PlanKey key = zkey(kind, m, n, nrhs, z);
  auto hp = host_plan(key);
  if (!hp->valid) return TQR_E_INTERNAL;
  const size_t tb = align_up(ztau_bytes(m, n, z.nb));
  if (w_bytes < tb + state_bytes((int64_t)hp->g.tasks.size())) return TQR_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  DevicePlan dp;
  int rc = device_plan(key, *hp, dev, &dp);
  if (rc) return rc;
  int grid = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_z_grid.find({dev, z.nb});
    if (it != g_z_grid.end()) grid = it->second;
  }
  if (!grid) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    grid = cus * zqr_occupancy(z.nb);
    std::lock_guard<std::mutex> lk(g_mu);
    g_z_grid[{dev, z.nb}] = grid;
  }
  char *w = static_cast<char *>(W);
  ExecArgs a{};
  set_plan(a, dp);
  a.ctl = reinterpret_cast<ExecCtl *>(w + tb);
  a.queue = reinterpret_cast<int32_t *>(w + tb + align_up(sizeof(ExecCtl)));
  a.indeg = reinterpret_cast<int32_t *>(w + tb + align_up(sizeof(ExecCtl)) +
                                        align_up((size_t)std::max<int32_t>(a.ntasks, 1) * 4));
  // the complex matrices are passed as double pointers to interleaved
  // (re, im) pairs; leading dimensions count complex entries; Tf holds tau
  a.prob.A = static_cast<double *>(A);
  a.prob.lda = lda;
  a.prob.m = m;
  a.prob.n = n;
  a.prob.B = static_cast<double *>(B);
  a.prob.ldb = ldb;
  a.prob.nrhs = nrhs;
  a.prob.Tf = reinterpret_cast<double *>(w);
  a.prob.p = key.p;
  a.prob.q = key.q;
  a.prob.singular = &a.ctl->pad[0];
  a.nb = z.nb;
  a.spin_limit = spin_limit_ticks(dev);
  a.trace = g_trace;
  a.trace_cap = g_trace_cap;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (g_timing && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess)
    hipEventRecord(ev0, stream);
  const hipError_t e = launch_zqr(a, z.nb, grid, info, stream);
  if (ev1) {
    hipEventRecord(ev1, stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_events.emplace_back(ev0, ev1);
  }
  return e == hipSuccess ? TQR_OK : TQR_E_HIP;
}

}  // namespace

extern "C" {

size_t tqr_zworkspace_size(int64_t m, int64_t n, int64_t nrhs, const tqr_opts *o) {
  if (m < 1 || n < 1 || n > m || nrhs < 0) return 0;
  ZResolved z;
  if (zresolve(o, &z)) return 0;
  return zwork_bytes(m, n, nrhs, z);
}

int tqr_zfactor(int64_t m, int64_t n, void *A, int64_t lda, void *W, size_t w_bytes, const tqr_opts *o,
                int32_t *info, hipStream_t stream) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!W) return -5;
  ZResolved z;
  int rc = zresolve(o, &z);
  if (rc) return rc;
  return zrun(PK_ZFACTOR, m, n, A, lda, nullptr, 0, 0, W, w_bytes, z, info, stream);
}

int tqr_zapply_qh(int64_t m, int64_t n, const void *A, int64_t lda, void *W, size_t w_bytes, int64_t nrhs, void *B,
                  int64_t ldb, const tqr_opts *o, int32_t *info, hipStream_t stream) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!W) return -5;
  if (nrhs < 1) return -7;
  if (!B) return -8;
  if (ldb < m) return -9;
  ZResolved z;
  int rc = zresolve(o, &z);
  if (rc) return rc;
  return zrun(PK_ZAPPLY, m, n, const_cast<void *>(A), lda, B, ldb, nrhs, W, w_bytes, z, info, stream);
}

// ------------------------------------------------ tile Cholesky inversion
}  // extern "C"

namespace {

PlanKey cholinv_key(int64_t n, int nb, int variant) {
  PlanKey k{};
  k.kind = PK_CHOLINV;
  k.p = k.q = (int)cdiv(n, nb);
  k.family = variant & TQR_CHOLINV_RENAMED ? 1 : 0;
  k.tree = variant & TQR_CHOLINV_UUU ? 1 : 0;
  k.stripes = k.stripes_b = 1;
  // the static list order (tab units as durations) for the in-place graph
  // (4096^2, nb 64: 26.7 -> 24.3 ms), the dynamic queue for the renamed one
  // (21.8 ms, 22.8 in the static order)
  if (k.family == 0) {
    k.priority = TQR_PRIO_STATIC;
    k.nb = nb;
    k.P = device_cus() * cholinv_occupancy(nb);
  } else {
    k.priority = TQR_PRIO_BOTTOM;
  }
  return k;
}

struct CholLayout {
  size_t state, l0, w0, total;
};

CholLayout cholinv_layout(int64_t n, int nb, int variant) {
  CholLayout L{};
  const int64_t nt = (int64_t)host_plan(cholinv_key(n, nb, variant))->g.tasks.size();
  L.state = 0;
  size_t off = align_up(state_bytes(nt));
  if (variant & TQR_CHOLINV_RENAMED) {
    L.l0 = off;
    off += align_up((size_t)n * n * 8);
    L.w0 = off;
    off += align_up((size_t)n * n * 8);
  }
  L.total = off;
  return L;
}

std::map<std::pair<int, int>, int> g_chol_grid;

}  // namespace

extern "C" {

size_t tqr_cholinv_work_size(int64_t n, int32_t nb, int32_t variant) {
  if (n < 1 || !cholinv_nb_supported(nb) || variant < 0 || variant > 3) return 0;
  return cholinv_layout(n, nb, variant).total;
}

int tqr_cholinv(int64_t n, double *A, int64_t lda, int32_t nb, int32_t variant, void *work, size_t work_bytes,
                int32_t *info, hipStream_t stream) {
  if (n < 1) return -1;
  if (!A) return -2;
  if (lda < n) return -3;
  if (!cholinv_nb_supported(nb)) return -4;
  if (variant < 0 || variant > 3) return -5;
  if (!work) return -6;
  const PlanKey key = cholinv_key(n, nb, variant);
  auto hp = host_plan(key);
  if (!hp->valid) return TQR_E_INTERNAL;
  const CholLayout L = cholinv_layout(n, nb, variant);
  if (work_bytes < L.total) return TQR_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  DevicePlan dp;
  int rc = device_plan(key, *hp, dev, &dp);
  if (rc) return rc;
  int grid = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_chol_grid.find({dev, nb});
    if (it != g_chol_grid.end()) grid = it->second;
  }
  if (!grid) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    grid = cus * cholinv_occupancy(nb);
    std::lock_guard<std::mutex> lk(g_mu);
    g_chol_grid[{dev, nb}] = grid;
  }
  char *w = static_cast<char *>(work);
  ExecArgs a{};
  set_plan(a, dp);
  a.ctl = reinterpret_cast<ExecCtl *>(w + L.state);
  a.queue = reinterpret_cast<int32_t *>(w + L.state + align_up(sizeof(ExecCtl)));
  a.indeg = reinterpret_cast<int32_t *>(w + L.state + align_up(sizeof(ExecCtl)) +
                                        align_up((size_t)std::max<int32_t>(a.ntasks, 1) * 4));
  a.prob.A = A;
  a.prob.lda = lda;
  a.prob.m = n;
  a.prob.n = n;
  // copies of L and L^{-1} (renamed variant): the tile kernels take them from
  // the Problem's B and Tf pointers, leading dimension ldb
  a.prob.B = (variant & TQR_CHOLINV_RENAMED) ? reinterpret_cast<double *>(w + L.l0) : nullptr;
  a.prob.Tf = (variant & TQR_CHOLINV_RENAMED) ? reinterpret_cast<double *>(w + L.w0) : nullptr;
  a.prob.ldb = n;
  a.prob.p = a.prob.q = key.p;
  a.prob.singular = &a.ctl->pad[0];
  a.nb = nb;
  a.spin_limit = spin_limit_ticks(dev);
  a.trace = g_trace;
  a.trace_cap = g_trace_cap;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (g_timing && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess)
    hipEventRecord(ev0, stream);
  const hipError_t e = launch_cholinv(a, nb, grid, info, stream);
  if (ev1) {
    hipEventRecord(ev1, stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_events.emplace_back(ev0, ev1);
  }
  return e == hipSuccess ? TQR_OK : TQR_E_HIP;
}

int tqr_cholinv_graph_stats(int32_t t, int32_t variant, int64_t *ntasks, double *cp_tasks, double *cp_weighted) {
  if (t < 1) return -1;
  if (variant < 0 || variant > 3) return -2;
  const bool inplace = !(variant & TQR_CHOLINV_RENAMED), udu = !(variant & TQR_CHOLINV_UUU);
  Graph gw = build_cholinv_graph(t, inplace, udu, false);
  Graph gu = build_cholinv_graph(t, inplace, udu, true);
  finalize(gw, true);
  if (!validate(gw)) return TQR_E_INTERNAL;
  if (ntasks) *ntasks = (int64_t)gw.tasks.size();
  if (cp_tasks) *cp_tasks = gu.cp;
  if (cp_weighted) *cp_weighted = gw.cp;
  return TQR_OK;
}

int tqr_schedule_bounds(int64_t m, int64_t n, const tqr_opts *o, int32_t P, double *out) {
  if (m < 1) return -1;
  if (n < 1 || n > m) return -2;
  if (P < 1) return -4;
  if (!out) return -5;
  Resolved r;
  int rc = resolve(o, &r, m, n);
  if (rc) return rc;
  // a fresh graph: the cached plans drop their predecessor lists
  const PlanKey k = make_key(PK_FACTOR, (int)cdiv(m, r.nb), (int)cdiv(n, r.nb), 0, r);
  GraphSpec spec;
  spec.p = k.p;
  spec.q = k.q;
  spec.family = k.family;
  spec.stripes = k.stripes;
  Graph g = build_graph(make_list(k.tree, k.p, k.q, k.param), spec);
  finalize(g, true);
  if (!validate(g)) return TQR_E_INTERNAL;
  double tseq = 0.0;
  for (double w : g.weight) tseq += w;
  out[0] = g.cp;
  out[1] = tseq;
  out[2] = alap_lost_area(g, P);
  out[3] = alap_bound(g, P);
  out[4] = list_makespan(g, P);
  return TQR_OK;
}

void tqr_debug_timing(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &pr : g_events) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  g_events.clear();
  g_timing = enable != 0;
}

int tqr_debug_timing_read(double *ms_total, int64_t *launches) {
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0.0;
  for (auto &pr : g_events) {
    if (hipEventSynchronize(pr.second) != hipSuccess) return TQR_E_HIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return TQR_E_HIP;
    tot += ms;
  }
  if (ms_total) *ms_total = tot;
  if (launches) *launches = (int64_t)g_events.size();
  return TQR_OK;
}

int tqr_executor_grid(const tqr_opts *o) {
  Resolved r;
  const int rc = resolve(o, &r);
  if (rc) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  return grid_size(dev, r.nb, r.ib);
}

int64_t tqr_wallclock_khz(void) {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TQR_E_HIP;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return TQR_E_HIP;
  return khz;
}

void tqr_debug_spin_limit(int64_t ticks) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_spin_override = ticks > 0 ? ticks : 0;
}

void tqr_debug_trace(int64_t *buf, int64_t cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_trace = buf;
  g_trace_cap = buf ? cap : 0;
}

}  // extern "C"

namespace {
// The plan the debug exports describe: a QR plan (kinds 0-5), or with kind
// 6 the Cholesky inversion of order m = n, tile size o->nb and variant
// o->param.
int debug_key(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o, PlanKey *key) {
  if (m < 1 || n < 1 || n > m) return -1;
  if (kind == PK_CHOLINV) {
    if (m != n || !o || !cholinv_nb_supported(o->nb) || o->param < 0 || o->param > 3) return -5;
    *key = cholinv_key(n, o->nb, o->param);
    return TQR_OK;
  }
  if (kind < PK_FACTOR || kind > PK_SNE) return -4;
  Resolved r;
  const int rc = resolve(o, &r, m, n);
  if (rc) return rc;
  *key = make_key(kind, (int)cdiv(m, r.nb), (int)cdiv(n, r.nb), kind == PK_FACTOR ? 0 : nrhs, r);
  return TQR_OK;
}
}  // namespace

extern "C" {

int tqr_debug_graph(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o, int32_t *tasks,
                    int64_t cap) {
  PlanKey key{};
  const int rc = debug_key(m, n, nrhs, kind, o, &key);
  if (rc) return rc;
  auto hp = host_plan(key);
  const int64_t nt = (int64_t)hp->g.tasks.size();
  if (tasks && cap >= nt)
    for (int64_t t = 0; t < nt; t++) {
      const Task &x = hp->g.tasks[t];
      int32_t *o8 = tasks + 8 * t;
      o8[0] = x.kind;
      o8[1] = x.i;
      o8[2] = x.piv;
      o8[3] = x.k;
      o8[4] = x.j;
      o8[5] = x.stripe;
      o8[6] = hp->g.succ_off[t + 1] - hp->g.succ_off[t];
      o8[7] = hp->g.indeg0[t];
    }
  return (int)nt;
}

int tqr_debug_succ(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o, int32_t *off,
                   int32_t *succ, int64_t cap) {
  PlanKey key{};
  const int rc = debug_key(m, n, nrhs, kind, o, &key);
  if (rc) return rc;
  auto hp = host_plan(key);
  if ((int64_t)hp->g.succ.size() > cap) return -1;
  std::copy(hp->g.succ_off.begin(), hp->g.succ_off.end(), off);
  std::copy(hp->g.succ.begin(), hp->g.succ.end(), succ);
  return (int)hp->g.succ.size();
}

int tqr_debug_ready(int64_t m, int64_t n, int64_t nrhs, int32_t kind, const tqr_opts *o, int32_t *ready,
                    int64_t cap) {
  PlanKey key{};
  const int rc = debug_key(m, n, nrhs, kind, o, &key);
  if (rc) return rc;
  auto hp = host_plan(key);
  const Graph &g = hp->g;
  if ((int64_t)g.ready0.size() > cap) return -1;
  std::copy(g.ready0.begin(), g.ready0.end(), ready);
  return (int)g.ready0.size();
}

const char *tqr_strerror(int code) {
  switch (code) {
    case TQR_OK: return "ok";
    case TQR_E_HIP: return "a HIP call failed";
    case TQR_E_WORKSPACE: return "workspace too small";
    case TQR_E_UNSUPPORTED: return "unsupported option combination";
    case TQR_E_NOMEM: return "out of device memory for task tables";
    case TQR_E_INTERNAL: return "task graph failed validation";
    case TQR_E_SCRATCH:
      return "problem too large for the allocation-free entry point's scratch (TQR_NOALLOC_SCRATCH_BYTES)";
    case TQR_INFO_TIMEOUT: return "device executor watchdog fired";
    case TQR_INFO_NOCONV: return "refinement did not converge";
    default: return code < 0 ? "illegal argument" : "R has an exactly zero diagonal entry";
  }
}

}  // extern "C"
