"""Near-critical task marks (bit 28 of the kind word, planner side, CPU).

The planner marks the tasks whose slack in its dispatch cost model (the
critical path minus the longest path through the task) is under half a
single product; the device raises their waves' issue priority.  The marks
change the schedule only, never a result (the executor tests and the GPU
parity tests run plans that carry them).  A task of zero slack has a
predecessor of zero slack unless it is a source, and a successor of zero
slack unless it is a sink, so the marked set holds a whole source-to-sink
path: the critical path of the model."""
import numpy as np
import pytest

import paper_1002_4057_amd as spd

URGENT = 1 << 28
POTRF = 2


def succ_lists(p):
    tasks, succ = p["tasks"], p["succ"]
    return [succ[tasks[v, 6]:tasks[v, 7]].tolist() for v in range(len(tasks))]


@pytest.mark.parametrize("t,workers,opts", [(8, 64, {}), (16, 64, {}), (32, 256, dict(chain=1)),
                                             (24, 128, dict(renamed=0, trtri_first=1)),
                                             (16, 64, dict(loop_order=1)), (12, 64, dict(steps=1))])
def test_marks_hold_a_critical_path(t, workers, opts):
    p = spd.plan_export(t, workers=workers, **opts)
    code = p["tasks"][:, 0]
    urgent = (code & URGENT) != 0
    n = len(code)
    assert 0 < urgent.sum() < n / 2
    sl = succ_lists(p)
    has_pred = np.zeros(n, bool)
    for v in range(n):
        for s in sl[v]:
            has_pred[s] = True
    # a path of marked tasks from a source to a sink (program order is
    # topological: one pass in order propagates reachability)
    reach = urgent & ~has_pred
    for v in range(n):
        if reach[v]:
            for s in sl[v]:
                if urgent[s]:
                    reach[s] = True
    sinks = np.array([len(x) == 0 for x in sl])
    assert np.any(reach & sinks)
    # the barrier tasks (no work) are never marked; the step-1 chain of
    # POTRFs mostly is
    assert not np.any(urgent & ((code & 0xFF) == 0))
    potrf = (code & 0xFF) == POTRF
    assert urgent[potrf].mean() > 0.5

