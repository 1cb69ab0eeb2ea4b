"""The executor's ready queue and its static list order, checked on the CPU.

* The static order (TQR_PRIO_STATIC, the default): every task of the graph
  exactly once, each after all its predecessors, starting with the first
  panel; the one-queue orders list only the initially ready tasks.
* A step-by-step model of the device protocol (exec_loop.h: a workgroup
  takes the next slot, polls it with relaxed loads until it holds a task
  whose predecessors have all finished, runs it, then decrements its
  successors' counts and pushes those that reach zero, except with the
  static order, whose queue is filled from the start), run with random
  interleavings of every shared memory access over real task graphs: every
  task runs exactly once, after all its predecessors finished, and every
  workgroup exits (no deadlock, no early exit).  A planted mistake in the
  model fails the same checks.
"""
import random

import numpy as np
import pytest

import paper_1303_3182_amd as T

NB = 128


def _graph(m, n, tree, kernels, priority, kind=3, nrhs=1):
    o = T.default_opts(nb=NB, ib=32, tree=tree, kernels=kernels, priority=priority)
    tasks = T.debug_graph(m, n, o, nrhs=nrhs, kind=kind)
    off, succ = T.debug_succ(m, n, o, nrhs=nrhs, kind=kind)
    ready = T.debug_ready(m, n, o, nrhs=nrhs, kind=kind)
    return tasks, off, succ, ready


def test_static_order_lists_every_task_after_its_predecessors():
    for (tree, kernels, shape) in [("flat", "hybrid", (12, 12)), ("greedy", "tt", (16, 4)),
                                   ("fibonacci", "hybrid", (9, 5))]:
        m, n = shape[0] * NB, shape[1] * NB
        tasks, off, succ, ready = _graph(m, n, tree, kernels, "static")
        assert sorted(ready) == list(range(len(tasks)))
        pos = np.empty(len(tasks), dtype=np.int64)
        pos[np.array(ready)] = np.arange(len(tasks))
        for t in range(len(tasks)):
            for e in range(off[t], off[t + 1]):
                assert pos[succ[e]] > pos[t]
        # a list schedule starts with a panel kernel of tile column 0
        assert tasks[ready[0]][0] in (0, 1, 2) and tasks[ready[0]][3] == 0


def test_one_queue_orders_list_the_initially_ready_tasks():
    m, n = 10 * NB, 6 * NB
    tasks, off, succ, ready_s = _graph(m, n, "greedy", "tt", "static")
    indeg = np.zeros(len(tasks), dtype=np.int64)
    for s in succ:
        indeg[s] += 1
    for pr in ("bottom", "list"):
        t2, off2, succ2, ready = _graph(m, n, "greedy", "tt", pr)
        assert t2 == tasks and off2 == off and sorted(succ2) == sorted(succ)
        assert sorted(ready) == sorted(np.flatnonzero(indeg == 0).tolist())


def _simulate(ntasks, off, succ, ready, workgroups, rng, static=False, planted=None,
              max_steps=3_000_000):
    """Runs the device protocol with `workgroups` workgroups, one shared
    memory access per step, the next workgroup to step drawn at random.
    Returns the order in which tasks started.  static: the queue holds every
    task from the start and a finished task pushes nothing.  planted: a
    planted mistake, "exit" (a workgroup that finds its slot not yet ready
    leaves) or "no-wait" (a slot's task starts without its predecessor
    count reaching zero)."""
    indeg0 = np.zeros(ntasks, dtype=np.int64)
    for s in succ:
        indeg0[s] += 1
    preds_left = indeg0.copy()
    queue = [-1] * ntasks
    for x, t in enumerate(ready):
        queue[x] = t
    S = {"head": 0, "tail": len(ready)}
    indeg = indeg0.copy()
    state = np.zeros(ntasks, dtype=np.int64)  # 0 waiting, 1 running, 2 done
    started = []

    def wg():
        while True:
            h = S["head"]
            S["head"] += 1
            yield
            if h >= ntasks:
                return
            while True:
                t = queue[h]
                yield
                if t >= 0 and (indeg[t] == 0 or planted == "no-wait"):
                    break
                if planted == "exit":
                    return
                yield
            assert state[t] == 0, "task %d started twice" % t
            assert preds_left[t] == 0, "task %d started before a predecessor ended" % t
            state[t] = 1
            started.append(t)
            for _ in range(rng.randrange(1, 8)):
                yield
            state[t] = 2
            for e in range(off[t], off[t + 1]):
                s = succ[e]
                preds_left[s] -= 1
                indeg[s] -= 1
                if indeg[s] == 0 and not static:
                    q = S["tail"]
                    S["tail"] += 1
                    yield
                    queue[q] = s
                yield

    gens = [wg() for _ in range(workgroups)]
    live = list(range(workgroups))
    steps = 0
    while live:
        i = rng.randrange(len(live))
        try:
            next(gens[live[i]])
        except StopIteration:
            live.pop(i)
        steps += 1
        assert steps < max_steps, "no progress: the protocol deadlocked"
    assert (state == 2).all(), "a workgroup exited before every task ran"
    return started


@pytest.mark.parametrize("priority", ["bottom", "static"])
@pytest.mark.parametrize("tree,kernels,shape", [("flat", "hybrid", (6, 6)), ("greedy", "tt", (8, 3)),
                                                ("fibonacci", "hybrid", (7, 4))])
@pytest.mark.parametrize("workgroups", [1, 3, 16])
def test_protocol_on_library_graphs(priority, tree, kernels, shape, workgroups):
    m, n = shape[0] * NB, shape[1] * NB
    tasks, off, succ, ready = _graph(m, n, tree, kernels, priority)
    rng = random.Random(hash((priority, tree, shape, workgroups)) & 0xffff)
    started = _simulate(len(tasks), off, succ, ready, workgroups, rng, static=priority == "static")
    assert sorted(started) == list(range(len(tasks)))
    if priority == "static" and workgroups == 1:
        assert started == ready  # one workgroup runs the order as given


@pytest.mark.parametrize("planted", ["exit", "no-wait"])
def test_model_catches_planted_mistakes(planted):
    """Each planted mistake fails the model's checks; the same graph and
    interleavings pass with the protocol as built."""
    m, n = 6 * NB, 6 * NB
    tasks, off, succ, ready = _graph(m, n, "flat", "hybrid", "static")
    with pytest.raises(AssertionError, match="exited before every task ran|before a predecessor ended"):
        _simulate(len(tasks), off, succ, ready, 4, random.Random(3), static=True, planted=planted)
    started = _simulate(len(tasks), off, succ, ready, 4, random.Random(3), static=True)
    assert sorted(started) == list(range(len(tasks)))
