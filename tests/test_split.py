"""Row-half split of the step-1 critical path (planner side, CPU).

Between POTRF(j) and POTRF(j+1) the DAG runs TRSM(j+1, j) and then the last
SYRK into tile (j+1, j+1) (Alg. 1, step 1).  With several workers the
planner runs each of them as two row-half tasks (bits 24/25 of the kind
word); these tests check which tasks are split and that the halves carry
the whole product's dependencies.  The executor tests (schedule fuzzing)
run the split plans in random orders against the oracle.
"""
import numpy as np
import pytest

import paper_1002_4057_amd as spd

HALF, HALF_HI = 1 << 24, 1 << 25
SYRK1, POTRF, TRSM1 = 1, 2, 4


def preds_of(p):
    tasks, succ = p["tasks"], p["succ"]
    pr = [set() for _ in range(len(tasks))]
    for v in range(len(tasks)):
        for s in succ[tasks[v, 6]:tasks[v, 7]]:
            pr[int(s)].add(v)
    return pr


@pytest.mark.parametrize("opts", [dict(), dict(chain=1), dict(renamed=0), dict(pipelined=0)])
@pytest.mark.parametrize("t", [2, 3, 6, 9])
def test_split_marks_the_step1_path(t, opts):
    p = spd.plan_export(t, workers=8, **opts)
    tasks = p["tasks"]
    code = tasks[:, 0]
    kind = code & 0xFF
    half = (code & HALF) != 0
    hi = (code & HALF_HI) != 0
    assert not np.any(hi & ~half)
    lo_idx = np.where(half & ~hi)[0]
    hi_idx = np.where(hi)[0]
    # one TRSM and one SYRK per step from POTRF(j) to POTRF(j+1)
    assert len(lo_idx) == len(hi_idx) == 2 * (t - 1)
    assert sorted(kind[lo_idx].tolist()) == [SYRK1] * (t - 1) + [TRSM1] * (t - 1)
    pr = preds_of(p)
    succ = p["succ"]
    for u in lo_idx:
        v = u + 1                                   # the second half follows the first
        assert hi[v] and np.array_equal(tasks[u, 1:6], tasks[v, 1:6])
        assert (code[u] | HALF_HI) == code[v]
        assert tasks[u, 0] & (0xF << 20) == 0       # single products only
        assert pr[u] == pr[v]                       # same predecessors
        su = set(succ[tasks[u, 6]:tasks[u, 7]].tolist())
        sv = set(succ[tasks[v, 6]:tasks[v, 7]].tolist())
        assert su == sv and len(su) > 0             # every successor waits for both
    potrf = np.where(kind == POTRF)[0]
    for j in range(1, t):
        v = potrf[j]
        sy = [u for u in pr[v] if kind[u] == SYRK1]
        assert len(sy) == 2 and all(half[u] for u in sy)      # the last SYRK, in halves
        assert all(tasks[u, 1] == tasks[v, 1] for u in sy)
        tr = [u for u in pr[sy[0]] if kind[u] == TRSM1]
        assert len(tr) == 2 and all(half[u] for u in tr)      # TRSM(j, j-1), in halves
        assert all(tasks[u, 1] == tasks[sy[0], 2] for u in tr)


@pytest.mark.parametrize("t", [4, 7])
def test_no_split_with_one_worker_or_when_turned_off(t):
    for p in (spd.plan_export(t, workers=1), spd.plan_export(t, workers=8, no_split=1)):
        assert not np.any(p["tasks"][:, 0] & (HALF | HALF_HI))
    whole = spd.plan_export(t, workers=8, no_split=1)
    split = spd.plan_export(t, workers=8)
    assert len(split["tasks"]) == len(whole["tasks"]) + 2 * (t - 1)


@pytest.mark.parametrize("bad", [2, -1])
def test_split_option_range_checked(bad):
    """An out-of-range no_split is rejected before anything touches the device."""
    import ctypes
    from paper_1002_4057_amd import _lib
    lib = _lib.load()
    o = _lib.make_opts(no_split=bad)
    assert lib.spd_inverse(4, ctypes.c_void_p(8), 4, 0, None, 0, None, ctypes.byref(o), None,
                           None) != 0


@pytest.mark.parametrize("steps,s", [(9, 1), (9, 2), (8, 1)])
@pytest.mark.parametrize("t", [3, 6])
def test_solve_chain_products_split(t, steps, s):
    """In the solve each row's multiplication by D_i (or D_i^T) and the last
    update of that right-hand-side tile before it form the chain of
    dependent tasks; both run as row halves."""
    GEMMS, TRSMS = 13, 14
    p = spd.plan_export(t, workers=8, steps=steps, rhs_tiles=s)
    tasks = p["tasks"]
    code = tasks[:, 0]
    kind = code & 0xFF
    half, hi = (code & HALF) != 0, (code & HALF_HI) != 0
    trsms = np.where((kind == TRSMS) & ~hi)[0]
    assert len(trsms) == 2 * t * s and np.all(half[trsms])
    pr = preds_of(p)
    for v in trsms:
        ups = [u for u in pr[v] if kind[u] == GEMMS and tasks[u, 1] == tasks[v, 1]]
        assert all(half[u] for u in ups)
    n_hi = int(hi.sum())
    whole = spd.plan_export(t, workers=8, steps=steps, rhs_tiles=s, no_split=1)
    assert len(tasks) == len(whole["tasks"]) + n_hi
