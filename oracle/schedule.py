"""ORACLE -- test infrastructure only (see oracle/__init__).

Task graphs of tiled algorithms and their scheduling on a bounded number of
processors, written from the thesis's chapters "Scheduling of Cholesky
Factorization" and "Scheduling of QR Factorization":

* ``qr_dag``: the task graph of a tiled QR factorization driven by an
  elimination list (chapter "QR Factorization": algorithm alg.elimTR for TT
  kernels, alg.elimSQ for the hybrid TS/TT expansion), with the kernel
  weights of table tab.kernels.  Edges are the data-flow hazards on the
  separate items of each tile (the upper part holding R or a TT reflector,
  the lower part holding GEQRT's reflector, the two T factors, and each
  trailing tile), honoured in list order: read after write, write after
  read, write after write.
* ``cholesky_dag``: the task graph of the tile Cholesky factorization (step 1
  of algorithm alg:InPlace) with the weights of table tab:taskweights.
* ``bottom_levels``: the Backflow priorities (section "Critical Path
  Scheduling"): a task's priority is its own weight plus the largest
  priority among its successors.
* ``list_schedule``: the critical-path ("CP method") schedule on P
  processors: whenever a processor is idle it starts the ready task of
  largest priority; ties go to the task that became ready first, then to
  the task created last (the thesis does not state its tie rule; this one
  reproduces every cell of table tab:5x5_optimal except four that depend
  on it, and a misprint).
* ``alap_bound``: the ALAP derived performance bound (equation
  eqn:alapbound): every task starts as late as possible on unbounded
  processors; LA_P is the idle area of P processors over the tail of that
  execution in which it never uses more than P of them; the bound is
  T_P = (T_seq + LA_P) / P, and never below the critical path.

Weights are integers, so times are integers and every profile is a step
function on unit slots.
"""
from fractions import Fraction
import heapq

QR_WEIGHTS = {"GEQRT": 4, "TSQRT": 6, "TTQRT": 2, "UNMQR": 6, "TSMQR": 12, "TTMQR": 6}
CHOL_WEIGHTS = {"POTRF": 1, "TRSM": 3, "SYRK": 3, "GEMM": 6}


class Dag:
    """Tasks in creation order: name (a tuple), weight, predecessor set."""

    def __init__(self):
        self.names = []
        self.w = []
        self.preds = []
        self._last_writer = {}
        self._readers = {}

    def add(self, name, weight, reads=(), writes=()):
        """Adds a task that reads `reads` and reads-and-writes `writes`;
        its predecessors follow from the hazards on those items."""
        t = len(self.names)
        pr = set()
        for it in list(reads) + list(writes):
            if it in self._last_writer:
                pr.add(self._last_writer[it])          # read / write after write
        for it in writes:
            pr.update(self._readers.get(it, ()))       # write after read
        pr.discard(t)
        self.names.append(name)
        self.w.append(weight)
        self.preds.append(pr)
        for it in reads:
            self._readers.setdefault(it, []).append(t)
        for it in writes:
            self._last_writer[it] = t
            self._readers[it] = []
        return t

    def succs(self):
        s = [[] for _ in self.names]
        for t, pr in enumerate(self.preds):
            for u in sorted(pr):
                s[u].append(t)
        return s

    def total_work(self):
        return sum(self.w)


def qr_dag(p, q, elist, mode="tt"):
    """Task graph of the tiled QR of p x q tiles for an elimination list of
    (i, piv, k) triples (1-based).  mode "tt": algorithm alg.elimTR (every
    tile of column 1 triangularised first; a row killed in column k < q is
    triangularised in column k+1).  mode "hybrid": a pivot is triangularised
    at its first use in a column, a killed square tile is killed by
    TSQRT/TSMQR, a killed triangle by TTQRT/TTMQR (alg.elimSQ mixed with
    alg.elimTR)."""
    d = Dag()
    W = QR_WEIGHTS
    tri = set()

    def geqrt(i, k):
        d.add(("GEQRT", i, k), W["GEQRT"], reads=[("C", i, k)],
              writes=[("U", i, k), ("L", i, k), ("TG", i, k)])
        tri.add((i, k))
        for j in range(k + 1, q + 1):
            d.add(("UNMQR", i, k, j), W["UNMQR"], reads=[("L", i, k), ("TG", i, k)], writes=[("C", i, j)])

    def kill(i, piv, k, ts):
        if ts:
            d.add(("TSQRT", i, piv, k), W["TSQRT"], reads=[("C", i, k)],
                  writes=[("U", piv, k), ("U", i, k), ("L", i, k), ("TK", i, k)])
            for j in range(k + 1, q + 1):
                d.add(("TSMQR", i, piv, k, j), W["TSMQR"], reads=[("U", i, k), ("L", i, k), ("TK", i, k)],
                      writes=[("C", piv, j), ("C", i, j)])
        else:
            d.add(("TTQRT", i, piv, k), W["TTQRT"], writes=[("U", piv, k), ("U", i, k), ("TK", i, k)])
            for j in range(k + 1, q + 1):
                d.add(("TTMQR", i, piv, k, j), W["TTMQR"], reads=[("U", i, k), ("TK", i, k)],
                      writes=[("C", piv, j), ("C", i, j)])

    if mode == "tt":
        for i in range(1, p + 1):
            geqrt(i, 1)
        for (i, piv, k) in elist:
            kill(i, piv, k, ts=False)
            if k < q:
                geqrt(i, k + 1)
    elif mode == "hybrid":
        for (i, piv, k) in elist:
            if (piv, k) not in tri:
                geqrt(piv, k)
            kill(i, piv, k, ts=(i, k) not in tri)
        if p == q and (q, q) not in tri:
            geqrt(q, q)
    else:
        raise ValueError(mode)
    return d


def cholesky_dag(t):
    """Task graph of the tile Cholesky factorization of t x t tiles (lower),
    in the loop order of step 1 of algorithm alg:InPlace: for each column j,
    the SYRKs into A(j,j), POTRF(j), the GEMMs into the tiles below it, then
    the TRSMs.  Tile (i,j) is one item updated in place."""
    d = Dag()
    W = CHOL_WEIGHTS
    for j in range(t):
        for k in range(j):
            d.add(("SYRK", j, k), W["SYRK"], reads=[(j, k)], writes=[(j, j)])
        d.add(("POTRF", j), W["POTRF"], writes=[(j, j)])
        for i in range(j + 1, t):
            for k in range(j):
                d.add(("GEMM", i, j, k), W["GEMM"], reads=[(i, k), (j, k)], writes=[(i, j)])
        for i in range(j + 1, t):
            d.add(("TRSM", i, j), W["TRSM"], reads=[(j, j)], writes=[(i, j)])
    return d


def bottom_levels(d):
    """Backflow priorities: bl(t) = w(t) + max over successors of bl (tasks
    are created in a topological order, so one reverse sweep suffices)."""
    s = d.succs()
    bl = [0] * len(d.w)
    for t in reversed(range(len(d.w))):
        bl[t] = d.w[t] + max((bl[u] for u in s[t]), default=0)
    return bl


def asap_times(d):
    """Start times with every task as soon as possible (unbounded processors)."""
    st = [0] * len(d.w)
    for t in range(len(d.w)):
        st[t] = max((st[u] + d.w[u] for u in d.preds[t]), default=0)
    return st


def critical_path(d):
    return max(bottom_levels(d), default=0)


def list_schedule(d, P, priority=None):
    """Makespan of the CP-method list schedule on P processors.

    Event driven: at each time, idle processors take ready tasks in order of
    decreasing priority (default: Backflow bottom level); equal priorities
    go to the task that became ready first, then to the one created last.
    Returns (makespan, start times)."""
    n = len(d.w)
    pri = bottom_levels(d) if priority is None else priority
    s = d.succs()
    npred = [len(pr) for pr in d.preds]
    ready = []  # heap of (-priority, ready time, -index)
    for t in range(n):
        if npred[t] == 0:
            heapq.heappush(ready, (-pri[t], 0, -t))
    running = []  # heap of (end, index)
    start = [None] * n
    time, idle, done = 0, P, 0
    while done < n:
        while idle > 0 and ready:
            _, _, mt = heapq.heappop(ready)
            t = -mt
            start[t] = time
            heapq.heappush(running, (time + d.w[t], t))
            idle -= 1
        time = running[0][0]
        while running and running[0][0] == time:
            _, t = heapq.heappop(running)
            idle += 1
            done += 1
            for u in s[t]:
                npred[u] -= 1
                if npred[u] == 0:
                    heapq.heappush(ready, (-pri[u], time, -u))
    return max(start[t] + d.w[t] for t in range(n)), start


def alap_profile(d):
    """Number of busy processors in each unit slot [x, x+1) of the ALAP
    execution on unbounded processors (start = cp - bottom level)."""
    bl = bottom_levels(d)
    cp = max(bl)
    prof = [0] * cp
    for t in range(len(d.w)):
        st = cp - bl[t]
        for x in range(st, st + d.w[t]):
            prof[x] += 1
    return prof


def lost_area(d, P):
    """LA_P: scanning the ALAP execution backwards from its end, the idle
    area of P processors until the first slot that needs more than P."""
    prof = alap_profile(d)
    la = 0
    for x in reversed(range(len(prof))):
        if prof[x] > P:
            break
        la += P - prof[x]
    return la


def alap_bound(d, P):
    """The ALAP derived bound T_P = max(cp, (T_seq + LA_P) / P), exact."""
    tseq = d.total_work()
    return max(Fraction(critical_path(d)), Fraction(tseq + lost_area(d, P), P))


# ------------------------------------------------- tile Cholesky inversion
CHOLINV_WEIGHTS = {"POTRF": 1, "TRSM": 3, "SYRK": 3, "GEMM": 6, "TRTRI": 1, "TRMM": 3, "LAUUM": 1}


def cholinv_dag(t, inplace=True, order="UDU", pipelined=True, weights=None):
    """Task graph of the tile Cholesky inversion of t x t tiles (lower), in
    the loop order of algorithm alg:InPlace (chapter "Cholesky Inversion"):
    step 1 the tile Cholesky factorization, step 2 the inversion of L, step
    3 the product L^{-T} L^{-1}; tile (i,j) is one item updated in place.

    `order` gives the direction of the innermost loop of each step (the
    successive commutative GEMMs; section "Algorithmic study", loop
    reversal): U increasing, D decreasing.  inplace=False is the variant
    with array renaming: step 2 reads the tiles of L from a copy taken at
    the end of step 1 and step 3 those of L^{-1} from a copy taken at the
    end of step 2, so those reads carry no anti-dependence (the copies are
    not tasks).  pipelined=False separates the steps: every task of a step
    waits for every task of the step before.  weights: None counts tasks
    (unit weights, as table table:criticalpath does); CHOLINV_WEIGHTS gives
    flops in units of nb^3/3."""
    d = Dag()
    W = weights or {}

    def w(kind):
        return W.get(kind, 1)

    def loop(rng, o):
        return list(rng) if o == "U" else list(reversed(list(rng)))

    step_tasks = []
    barrier = set()
    # the value of tile (i,j) at the end of the previous step: (writer task)
    snapshot = {}

    def add(name, reads=(), writes=(), copied=()):
        t_ = d.add(name, w(name[0]), reads=reads, writes=writes)
        d.preds[t_].update(barrier)
        for it in copied:  # read from the renamed copy: true dependence only
            if it in snapshot:
                d.preds[t_].add(snapshot[it])
        d.preds[t_].discard(t_)
        step_tasks.append(t_)
        return t_

    def end_step():
        nonlocal barrier
        snapshot.clear()
        snapshot.update(d._last_writer)
        if not pipelined:
            barrier = set(step_tasks)
        step_tasks.clear()

    def rd(i, j):
        """(reads, copied) for a read of tile (i,j) of the previous step's
        result."""
        return ([], [(i, j)]) if not inplace else ([(i, j)], [])

    # step 1: tile Cholesky factorization
    for j in range(t):
        for k in loop(range(j), order[0]):
            add(("SYRK", j, k), reads=[(j, k)], writes=[(j, j)])
        add(("POTRF", j), writes=[(j, j)])
        for i in range(j + 1, t):
            for k in loop(range(j), order[0]):
                add(("GEMM", i, j, k), reads=[(i, k), (j, k)], writes=[(i, j)])
        for i in range(j + 1, t):
            add(("TRSM", i, j), reads=[(j, j)], writes=[(i, j)])
    end_step()
    # step 2: triangular inversion of L
    for j in reversed(range(t)):
        add(("TRTRI", j), writes=[(j, j)])
        for i in reversed(range(j + 1, t)):
            add(("TRMM", i, j, "L"), reads=[(i, i)], writes=[(i, j)])
            for k in loop(range(j + 1, i), order[1]):
                r_, c_ = rd(k, j)
                add(("GEMM", i, j, k), reads=[(i, k)] + r_, writes=[(i, j)], copied=c_)
            add(("TRMM", i, j, "R"), reads=[(j, j)], writes=[(i, j)])
    end_step()
    # step 3: product of the lower triangular matrices
    for i in range(t):
        for j in range(i):
            r_, c_ = rd(i, i)
            add(("TRMM", i, j, "T"), reads=r_, writes=[(i, j)], copied=c_)
        add(("LAUUM", i), writes=[(i, i)])
        for j in range(i):
            for k in loop(range(i + 1, t), order[2]):
                r1, c1 = rd(k, i)
                r2, c2 = rd(k, j)
                add(("GEMM", i, j, k), reads=r1 + r2, writes=[(i, j)], copied=c1 + c2)
        for k in loop(range(i + 1, t), order[2]):
            r_, c_ = rd(k, i)
            add(("SYRK", i, k), reads=r_, writes=[(i, i)], copied=c_)
    end_step()
    return d


def cholinv_step_cps(t, inplace=True, order="UDU"):
    """Critical path (in tasks) of each step alone: the graph of the steps
    separated, minus the path up to the previous step's end."""
    out = []
    prev = 0
    for s in range(3):
        d = cholinv_dag(t, inplace, order, pipelined=False)
        # tasks of steps <= s
        names = d.names
        cnt = _step_counts(t)
        upto = sum(cnt[:s + 1])
        sub = Dag()
        sub.names, sub.w = names[:upto], d.w[:upto]
        sub.preds = [set(p) for p in d.preds[:upto]]
        cp = critical_path(sub)
        out.append(cp - prev)
        prev = cp
    return out


def _step_counts(t):
    s1 = t + t * (t - 1) // 2 * 2 + t * (t - 1) * (t - 2) // 6
    s2 = t + t * (t - 1) + t * (t - 1) * (t - 2) // 6
    s3 = t + t * (t - 1) // 2 * 2 + t * (t - 1) * (t - 2) // 6
    return [s1, s2, s3]
