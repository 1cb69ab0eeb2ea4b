"""The executor-trace checker (host only) on hand-made traces: a consistent
trace passes, an unrun task and a successor that started before its
predecessor ended are both reported."""
import numpy as np

from tests.gpu_util import trace_violations

# diamond 0 -> {1, 2} -> 3
OFF = [0, 2, 3, 4, 4]
SUCC = [1, 2, 3, 3]


def _trace(rows):
    return np.array([[s, e, 0, 0] for s, e in rows], dtype=np.int64).ravel()


def test_consistent_trace_passes():
    assert trace_violations(OFF, SUCC, _trace([(1, 5), (5, 9), (6, 8), (9, 12)]), 4) == []


def test_early_successor_is_reported():
    bad = trace_violations(OFF, SUCC, _trace([(1, 5), (5, 9), (6, 8), (8, 12)]), 4)
    assert bad == [("order", 1, 3, 1)]
    assert trace_violations(OFF, SUCC, _trace([(1, 5), (5, 9), (6, 8), (8, 12)]), 4, slack=1) == []


def test_unrun_task_is_reported():
    bad = trace_violations(OFF, SUCC, _trace([(1, 5), (0, 0), (6, 8), (9, 12)]), 4)
    assert ("not run", 1) in bad
