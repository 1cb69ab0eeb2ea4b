/*
 * ORACLE -- test infrastructure only.  Nothing in the product library may
 * include, link or call this file; only tests/, the smoke check and the
 * bench's CPU-baseline leg use it.
 *
 * Plain, deliberately unoptimised C model of the thesis's tiled QR
 * *scheduling* layer (Bouwmeester 2012, chapter "QR Factorization"):
 *
 *   - elimination lists elim(i, piv(i,k), k) (section "Elimination lists"),
 *     1-based row/column indices as in the thesis;
 *   - the coarse-grain model (section "Coarse-grain algorithms"): one time
 *     unit per elimination regardless of row length;
 *   - the tiled model (section "Tiled algorithms"): every elimination is
 *     expanded into the six kernels of table tab.kernels with weights
 *     GEQRT 4, TSQRT 6, TTQRT 2, UNMQR 6, TSMQR 12, TTMQR 6 (unit nb^3/3),
 *     each kernel starting as soon as its inputs are ready (section
 *     "Execution schemes"), unbounded processors.
 *
 * Readings where the thesis is silent or garbled (each is checked against
 * the thesis's printed tables by the oracle's tests):
 *   R-BT  BinaryTree is only given by table tab.tiled(d): a binary reduction
 *         of the rows k..p of column k anchored at the diagonal row.
 *   R-FIB Fibonacci groups are counted inside column k, the bottom group is
 *         truncated, piv = i - z for a group of z rows.
 *   R-GR  In algorithm alg.tiled-greedy the number of new zeros is
 *         nZ_new = nZ(j) + floor((nT_new - nZ(j)) / 2), i.e. it uses the
 *         triangularised count of *this* step; the loop runs until column
 *         min(q, p-1) is finished.
 *   R-ASAP ASAP pairs the bottom 2s of the available rows (top half kills
 *         bottom half, in order); a pivot is busy for one TTQRT.
 *   R-DF  Data-flow items: the upper (R / TT-reflector) part and the lower
 *         (GEQRT reflector) part of a factored tile, each full trailing
 *         tile, and separate T storage for the GEQRT and the killing
 *         kernel.  Hazards RAW, WAR and WAW are honoured in list order.
 *   R-HY  HYBRID kernels: a row is triangularised (GEQRT) at its first use
 *         as a pivot in a column; a killed row that is still square is
 *         killed with TSQRT/TSMQR, a triangular one with TTQRT/TTMQR.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { T_FLAT = 0, T_BINARY = 1, T_FIBONACCI = 2, T_GREEDY = 3, T_GRASAP = 4,
       T_PLASMA = 5, T_ASAP = 6 };
enum { M_TT = 0, M_HYBRID = 1 };
enum { K_GEQRT = 0, K_TSQRT, K_TTQRT, K_UNMQR, K_TSMQR, K_TTMQR };

/* table tab.kernels */
static const int64_t WEIGHT[6] = {4, 6, 2, 6, 12, 6};

/* ------------------------------------------------------------------ lists */
typedef struct {
  int n, cap;
  int *i, *piv, *k;
} elist;

static void el_push(elist *l, int i, int piv, int k) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 256;
    l->i = (int *)realloc(l->i, sizeof(int) * l->cap);
    l->piv = (int *)realloc(l->piv, sizeof(int) * l->cap);
    l->k = (int *)realloc(l->k, sizeof(int) * l->cap);
  }
  l->i[l->n] = i;
  l->piv[l->n] = piv;
  l->k[l->n] = k;
  l->n++;
}

static void el_free(elist *l) {
  free(l->i);
  free(l->piv);
  free(l->k);
  memset(l, 0, sizeof(*l));
}

static int imin(int a, int b) { return a < b ? a : b; }
static int64_t lmax(int64_t a, int64_t b) { return a > b ? a : b; }

/* Sameh-Kuck / FlatTree: elim(i, k, k), i = k+1..p, for every column. */
static void gen_flat(int p, int q, elist *l) {
  for (int k = 1; k <= imin(p, q); k++)
    for (int i = k + 1; i <= p; i++) el_push(l, i, k, k);
}

/* BinaryTree (reading R-BT): rows r_0 = k .. r_{n-1} = p; at level l the
 * row r_d with d = 2^(l-1) mod 2^l is eliminated by r_{d - 2^(l-1)}. */
static void gen_binary(int p, int q, elist *l) {
  for (int k = 1; k <= imin(p, q); k++) {
    int n = p - k + 1;
    for (int half = 1; half < n; half *= 2)
      for (int d = half; d < n; d += 2 * half) el_push(l, k + d, k + d - half, k);
  }
}

/* Fibonacci scheme of order 1 (Modi-Clarke), reading R-FIB.
 * y(r) = least y with r <= y(y+1)/2 + 1; rows of a column with equal y are
 * zeroed at the same step, bottom groups first. */
static int fib_y(int r) {
  int y = 1;
  while (r > y * (y + 1) / 2 + 1) y++;
  return y;
}
static int fib_x(int p) {
  int x = 0;
  while (x * (x + 1) / 2 < p - 1) x++;
  return x;
}
static void gen_fibonacci(int p, int q, elist *l) {
  int x = fib_x(p);
  for (int k = 1; k <= imin(p, q); k++) {
    /* steps in increasing order: step value c1 = x - y + 1, i.e. y from
     * large (early) to small (late). */
    for (int y = x; y >= 1; y--) {
      int lo = -1, hi = -1; /* rows of column k with this y */
      for (int i = k + 1; i <= p; i++)
        if (fib_y(i - k + 1) == y) {
          if (lo < 0) lo = i;
          hi = i;
        }
      if (lo < 0) continue;
      int z = hi - lo + 1;
      for (int i = lo; i <= hi; i++) el_push(l, i, i - z, k);
    }
  }
}

/* Thesis's closed form for the Fibonacci coarse time steps:
 * coarse(i,1) = x - y + 1, and coarse(i,k) = coarse(i-1,k-1) + 2. */
static int fib_coarse(int p, int i, int k) {
  return fib_x(p) - fib_y(i - k + 1) + 1 + 2 * (k - 1);
}

/* Greedy, algorithm alg.tiled-greedy with reading R-GR. */
static void gen_greedy(int p, int q, elist *l) {
  int *nZ = (int *)calloc(q + 2, sizeof(int));
  int *nT = (int *)calloc(q + 2, sizeof(int));
  int last = imin(q, p - 1);
  while (last >= 1 && nZ[last] < p - last) {
    for (int j = q; j >= 1; j--) {
      int nTnew = (j == 1) ? p : nZ[j - 1];
      int nZnew = nZ[j] + (nTnew - nZ[j]) / 2;
      for (int kk = nZ[j]; kk < nZnew; kk++) {
        int row = p - kk;
        int piv = p - kk - nZnew + nZ[j];
        el_push(l, row, piv, j);
      }
      nT[j] = nTnew;
      nZ[j] = nZnew;
    }
  }
  free(nZ);
  free(nT);
}

/* PlasmaTree(BS): in column k the rows k..p form domains of BS rows
 * starting at row k (the last one truncated); a flat tree inside each
 * domain, then a binary tree over the domain heads. */
static void gen_plasma(int p, int q, int bs, elist *l) {
  if (bs < 1) bs = 1;
  for (int k = 1; k <= imin(p, q); k++) {
    for (int h = k; h <= p; h += bs)
      for (int i = h + 1; i <= imin(p, h + bs - 1); i++) el_push(l, i, h, k);
    int nh = (p - k) / bs + 1; /* number of heads */
    for (int half = 1; half < nh; half *= 2)
      for (int d = half; d < nh; d += 2 * half)
        el_push(l, k + d * bs, k + (d - half) * bs, k);
  }
}

/* ------------------------------------------------------- tiled simulator */
typedef struct {
  int64_t wr, rd; /* end of last write, latest end of a read since then */
} item;

typedef struct {
  int p, q, mode;
  item *C, *U, *L, *TG, *TK; /* p*q each, index (i-1)*q + (j-1) */
  unsigned char *tri;        /* tile (i,k) is triangular (HYBRID mode) */
  int64_t *zero_t;           /* end of the kernel that zeroed (i,k) */
  int64_t *geqrt_t;          /* end of GEQRT(i,k) */
  int64_t *upd_t;            /* end of the updates of elim(i,.,k) on column k+1 */
  int64_t cp;
  int64_t count[6];
} sim;

#define IDX(s, i, j) (((int64_t)(i) - 1) * (s)->q + ((j) - 1))

/* Runs one kernel: reads nr items, reads+writes nw items. */
static int64_t run(sim *s, int kind, item **rd, int nr, item **wr, int nw) {
  int64_t start = 0;
  for (int a = 0; a < nr; a++) start = lmax(start, rd[a]->wr);
  for (int a = 0; a < nw; a++) start = lmax(start, lmax(wr[a]->wr, wr[a]->rd));
  int64_t end = start + WEIGHT[kind];
  for (int a = 0; a < nr; a++) rd[a]->rd = lmax(rd[a]->rd, end);
  for (int a = 0; a < nw; a++) {
    wr[a]->wr = end;
    wr[a]->rd = 0;
  }
  s->cp = lmax(s->cp, end);
  s->count[kind]++;
  return end;
}

static void k_geqrt(sim *s, int i, int k) {
  item *r[1] = {&s->C[IDX(s, i, k)]};
  item *w[3] = {&s->U[IDX(s, i, k)], &s->L[IDX(s, i, k)], &s->TG[IDX(s, i, k)]};
  s->geqrt_t[IDX(s, i, k)] = run(s, K_GEQRT, r, 1, w, 3);
  s->tri[IDX(s, i, k)] = 1;
}
static void k_unmqr(sim *s, int i, int k, int j) {
  item *r[2] = {&s->L[IDX(s, i, k)], &s->TG[IDX(s, i, k)]};
  item *w[1] = {&s->C[IDX(s, i, j)]};
  run(s, K_UNMQR, r, 2, w, 1);
}
static void k_ttqrt(sim *s, int i, int piv, int k) {
  item *w[3] = {&s->U[IDX(s, piv, k)], &s->U[IDX(s, i, k)], &s->TK[IDX(s, i, k)]};
  s->zero_t[IDX(s, i, k)] = run(s, K_TTQRT, NULL, 0, w, 3);
}
static void k_ttmqr(sim *s, int i, int piv, int k, int j) {
  item *r[2] = {&s->U[IDX(s, i, k)], &s->TK[IDX(s, i, k)]};
  item *w[2] = {&s->C[IDX(s, piv, j)], &s->C[IDX(s, i, j)]};
  int64_t e = run(s, K_TTMQR, r, 2, w, 2);
  if (j == k + 1) s->upd_t[IDX(s, i, k)] = e;
}
static void k_tsqrt(sim *s, int i, int piv, int k) {
  item *r[1] = {&s->C[IDX(s, i, k)]};
  item *w[4] = {&s->U[IDX(s, piv, k)], &s->U[IDX(s, i, k)], &s->L[IDX(s, i, k)],
                &s->TK[IDX(s, i, k)]};
  s->zero_t[IDX(s, i, k)] = run(s, K_TSQRT, r, 1, w, 4);
}
static void k_tsmqr(sim *s, int i, int piv, int k, int j) {
  item *r[3] = {&s->U[IDX(s, i, k)], &s->L[IDX(s, i, k)], &s->TK[IDX(s, i, k)]};
  item *w[2] = {&s->C[IDX(s, piv, j)], &s->C[IDX(s, i, j)]};
  int64_t e = run(s, K_TSMQR, r, 3, w, 2);
  if (j == k + 1) s->upd_t[IDX(s, i, k)] = e;
}

static void sim_init(sim *s, int p, int q, int mode) {
  memset(s, 0, sizeof(*s));
  s->p = p;
  s->q = q;
  s->mode = mode;
  size_t n = (size_t)p * q;
  s->C = (item *)calloc(n, sizeof(item));
  s->U = (item *)calloc(n, sizeof(item));
  s->L = (item *)calloc(n, sizeof(item));
  s->TG = (item *)calloc(n, sizeof(item));
  s->TK = (item *)calloc(n, sizeof(item));
  s->tri = (unsigned char *)calloc(n, 1);
  s->zero_t = (int64_t *)calloc(n, sizeof(int64_t));
  s->geqrt_t = (int64_t *)calloc(n, sizeof(int64_t));
  s->upd_t = (int64_t *)calloc(n, sizeof(int64_t));
  if (mode == M_TT) {
    /* Algorithm alg.elimTR with k = 0: triangularise every tile of the
     * first column and apply the transformations to its row. */
    for (int i = 1; i <= p; i++) {
      k_geqrt(s, i, 1);
      for (int j = 2; j <= q; j++) k_unmqr(s, i, 1, j);
    }
  }
}

static void sim_free(sim *s) {
  free(s->C);
  free(s->U);
  free(s->L);
  free(s->TG);
  free(s->TK);
  free(s->tri);
  free(s->zero_t);
  free(s->geqrt_t);
  free(s->upd_t);
}

/* One elimination elim(i, piv, k). */
static void sim_elim(sim *s, int i, int piv, int k) {
  int q = s->q;
  if (s->mode == M_TT) {
    /* Algorithm alg.elimTR */
    k_ttqrt(s, i, piv, k);
    for (int j = k + 1; j <= q; j++) k_ttmqr(s, i, piv, k, j);
    if (k < q) {
      k_geqrt(s, i, k + 1);
      for (int j = k + 2; j <= q; j++) k_unmqr(s, i, k + 1, j);
    }
  } else {
    /* Reading R-HY (algorithm alg.elimSQ where the killed tile is square) */
    if (!s->tri[IDX(s, piv, k)]) {
      k_geqrt(s, piv, k);
      for (int j = k + 1; j <= q; j++) k_unmqr(s, piv, k, j);
    }
    if (s->tri[IDX(s, i, k)]) {
      k_ttqrt(s, i, piv, k);
      for (int j = k + 1; j <= q; j++) k_ttmqr(s, i, piv, k, j);
    } else {
      k_tsqrt(s, i, piv, k);
      for (int j = k + 1; j <= q; j++) k_tsmqr(s, i, piv, k, j);
    }
  }
}

static void sim_finish(sim *s) {
  /* The last diagonal tile of a square tile matrix has nothing below it; it
   * still has to be triangularised. */
  if (s->mode == M_HYBRID && s->p == s->q && !s->tri[IDX(s, s->q, s->q)])
    k_geqrt(s, s->q, s->q);
}

/* ASAP on column k (reading R-ASAP): needs GEQRT(r,k) end times, i.e. the
 * simulation of every elimination of the columns left of k. */
static void asap_column(sim *s, int k, elist *l) {
  int p = s->p;
  int64_t *g = (int64_t *)calloc(p + 1, sizeof(int64_t));
  int64_t *busy = (int64_t *)calloc(p + 1, sizeof(int64_t));
  char *alive = (char *)calloc(p + 1, 1);
  int *A = (int *)malloc(sizeof(int) * (p + 1));
  int nalive = 0;
  int64_t t = -1;
  for (int r = k; r <= p; r++) {
    g[r] = s->geqrt_t[IDX(s, r, k)];
    alive[r] = 1;
    nalive++;
    if (t < 0 || g[r] < t) t = g[r];
  }
  while (nalive > 1) {
    int na = 0;
    for (int r = k; r <= p; r++)
      if (alive[r] && g[r] <= t && busy[r] <= t) A[na++] = r;
    if (na >= 2) {
      int sh = na / 2;
      int *sel = A + (na - 2 * sh);
      for (int j = 0; j < sh; j++) {
        el_push(l, sel[sh + j], sel[j], k);
        busy[sel[j]] = t + WEIGHT[K_TTQRT];
        alive[sel[sh + j]] = 0;
        nalive--;
      }
    }
    int64_t nt = -1;
    for (int r = k; r <= p; r++) {
      if (!alive[r]) continue;
      if (g[r] > t && (nt < 0 || g[r] < nt)) nt = g[r];
      if (busy[r] > t && (nt < 0 || busy[r] < nt)) nt = busy[r];
    }
    if (nt < 0) break; /* cannot happen for a consistent state */
    t = nt;
  }
  free(g);
  free(busy);
  free(alive);
  free(A);
}

/* GrASAP(ia): Greedy on columns 1..q-ia, ASAP on the last ia columns
 * (definition def.grasap).  ia = q gives ASAP on every column. */
static void gen_grasap(int p, int q, int ia, elist *out) {
  elist g = {0};
  gen_greedy(p, q, &g);
  sim s;
  sim_init(&s, p, q, M_TT);
  for (int e = 0; e < g.n; e++)
    if (g.k[e] <= q - ia) {
      el_push(out, g.i[e], g.piv[e], g.k[e]);
      sim_elim(&s, g.i[e], g.piv[e], g.k[e]);
    }
  for (int k = (q - ia + 1 < 1 ? 1 : q - ia + 1); k <= imin(q, p - 1); k++) {
    int before = out->n;
    asap_column(&s, k, out);
    for (int e = before; e < out->n; e++) sim_elim(&s, out->i[e], out->piv[e], out->k[e]);
  }
  sim_free(&s);
  el_free(&g);
}

static int generate(int tree, int p, int q, int param, elist *l) {
  if (p < 1 || q < 1 || q > p) return -1;
  switch (tree) {
    case T_FLAT: gen_flat(p, q, l); break;
    case T_BINARY: gen_binary(p, q, l); break;
    case T_FIBONACCI: gen_fibonacci(p, q, l); break;
    case T_GREEDY: gen_greedy(p, q, l); break;
    case T_GRASAP: gen_grasap(p, q, param < 1 ? 1 : param, l); break;
    case T_PLASMA: gen_plasma(p, q, param, l); break;
    case T_ASAP: gen_grasap(p, q, q, l); break;
    default: return -2;
  }
  return 0;
}

/* ============================================================ C interface */

/* Elimination list of `tree` for a p x q tile matrix (param: BS for
 * PlasmaTree, i for GrASAP(i)).  Returns the list length; entries are
 * written only when cap is large enough. */
int orc_list(int tree, int p, int q, int param, int *oi, int *opiv, int *ok, int cap) {
  elist l = {0};
  int rc = generate(tree, p, q, param, &l);
  if (rc) return rc;
  if (l.n <= cap)
    for (int e = 0; e < l.n; e++) {
      oi[e] = l.i[e];
      opiv[e] = l.piv[e];
      ok[e] = l.k[e];
    }
  int n = l.n;
  el_free(&l);
  return n;
}

/* Tiled execution of a given list.  zero_t / geqrt_t / upd_t (p*q,
 * row-major, may be NULL) receive the end time of the kernel that zeroes /
 * triangularises each tile and of the update of column k+1 that follows
 * the zeroing of (i,k) (0 where none runs); counts[6] receives the kernel counts in the
 * order GEQRT, TSQRT, TTQRT, UNMQR, TSMQR, TTMQR.  Returns the critical
 * path length in units of nb^3/3. */
int64_t orc_tiled(int p, int q, int mode, int n, const int *li, const int *lpiv,
                  const int *lk, int64_t *zero_t, int64_t *geqrt_t, int64_t *upd_t,
                  int64_t *counts) {
  sim s;
  sim_init(&s, p, q, mode);
  for (int e = 0; e < n; e++) sim_elim(&s, li[e], lpiv[e], lk[e]);
  sim_finish(&s);
  size_t np = (size_t)p * q;
  if (zero_t) memcpy(zero_t, s.zero_t, np * sizeof(int64_t));
  if (geqrt_t) memcpy(geqrt_t, s.geqrt_t, np * sizeof(int64_t));
  if (upd_t) memcpy(upd_t, s.upd_t, np * sizeof(int64_t));
  if (counts) memcpy(counts, s.count, sizeof(s.count));
  int64_t cp = s.cp;
  sim_free(&s);
  return cp;
}

/* Convenience: list + tiled critical path of a tree. */
int64_t orc_tree_cp(int tree, int p, int q, int param, int mode) {
  elist l = {0};
  if (generate(tree, p, q, param, &l)) return -1;
  int64_t cp = orc_tiled(p, q, mode, l.n, l.i, l.piv, l.k, NULL, NULL, NULL, NULL);
  el_free(&l);
  return cp;
}

/* Coarse-grain execution of a list: one step per elimination, each as soon
 * as both rows are ready (their tiles left of column k zeroed) and neither
 * is busy in column k.  out (p*q row-major) receives the step at which tile
 * (i,k) is zeroed.  Returns the coarse critical path. */
int orc_coarse(int p, int q, int n, const int *li, const int *lpiv, const int *lk, int *out) {
  int *zero = (int *)calloc((size_t)(p + 1) * (q + 1), sizeof(int));
  int *use = (int *)calloc((size_t)(p + 1) * (q + 1), sizeof(int));
#define Z(i, k) zero[(i) * (q + 1) + (k)]
#define U_(i, k) use[(i) * (q + 1) + (k)]
  int cp = 0;
  for (int e = 0; e < n; e++) {
    int i = li[e], piv = lpiv[e], k = lk[e];
    int st = Z(i, k - 1);
    if (Z(piv, k - 1) > st) st = Z(piv, k - 1);
    if (U_(i, k) > st) st = U_(i, k);
    if (U_(piv, k) > st) st = U_(piv, k);
    st += 1;
    Z(i, k) = st;
    U_(i, k) = st;
    U_(piv, k) = st;
    if (st > cp) cp = st;
  }
  if (out)
    for (int i = 1; i <= p; i++)
      for (int k = 1; k <= q; k++) out[(i - 1) * q + (k - 1)] = Z(i, k);
#undef Z
#undef U_
  free(zero);
  free(use);
  return cp;
}

/* The thesis's Fibonacci time-step formula for every tile (i > k). */
void orc_fib_coarse(int p, int q, int *out) {
  for (int i = 1; i <= p; i++)
    for (int k = 1; k <= q; k++) out[(i - 1) * q + (k - 1)] = (i > k) ? fib_coarse(p, i, k) : 0;
}
