"""Row-part split of the chains of dependent products (planner side, CPU).

Between POTRF(j) and POTRF(j+1) the DAG runs TRSM(j+1, j) and then the last
SYRK into tile (j+1, j+1) (Alg. 1, step 1); the solve's substitutions are
chains of the same kind.  With several workers the planner runs each of
these products as row-part tasks (bit 24 of the kind word, part index in
bits 25-26, four quarters with bit 27, else two halves); these tests check
which tasks are split and that the parts carry the whole product's
dependencies.  The executor tests (schedule fuzzing) run the split plans in
random orders against the oracle.
"""
import numpy as np
import pytest

import paper_1002_4057_amd as spd

PART, PARTS4 = 1 << 24, 1 << 27
SYRK1, POTRF, TRSM1 = 1, 2, 4


def parts_of(code):
    """(is a part, part index, number of parts) per task."""
    part = (code & PART) != 0
    return part, (code >> 25) & 3, np.where(code & PARTS4, 4, 2)


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
    part, idx, nparts = parts_of(code)
    heads = np.where(part & (idx == 0))[0]
    k = int(nparts[heads[0]])
    assert k in (2, 4) and np.all(nparts[part] == k)
    # one TRSM and one SYRK per step from POTRF(j) to POTRF(j+1)
    assert len(heads) == 2 * (t - 1) and int(part.sum()) == k * len(heads)
    assert sorted(kind[heads].tolist()) == [SYRK1] * (t - 1) + [TRSM1] * (t - 1)
    pr = preds_of(p)
    succ = p["succ"]
    for u in heads:
        su = set(succ[tasks[u, 6]:tasks[u, 7]].tolist())
        assert tasks[u, 0] & (0xF << 20) == 0       # single products only
        assert len(su) > 0
        for c in range(1, k):                       # the parts follow each other
            v = u + c
            assert part[v] and idx[v] == c and np.array_equal(tasks[u, 1:6], tasks[v, 1:6])
            assert pr[u] == pr[v]                   # same predecessors
            assert set(succ[tasks[v, 6]:tasks[v, 7]].tolist()) == su   # every successor waits for all
    potrf = np.where(kind == POTRF)[0]
    for j in range(1, t):
        v = potrf[j]
        sy = [u for u in pr[v] if kind[u] == SYRK1]
        assert len(sy) == k and all(part[u] for u in sy)      # the last SYRK, in parts
        assert all(tasks[u, 1] == tasks[v, 1] for u in sy)
        tr = [u for u in pr[sy[0]] if kind[u] == TRSM1]
        assert len(tr) == k and all(part[u] for u in tr)      # TRSM(j, j-1), in parts
        assert all(tasks[u, 1] == tasks[sy[0], 2] for u in tr)


@pytest.mark.parametrize("t", [4, 7])
def test_no_split_with_one_worker_or_when_turned_off(t):
    for p in (spd.plan_export(t, workers=1), spd.plan_export(t, workers=8, no_split=1)):
        assert not np.any(p["tasks"][:, 0] & (PART | PARTS4 | (3 << 25)))
    whole = spd.plan_export(t, workers=8, no_split=1)
    split = spd.plan_export(t, workers=8)
    code = split["tasks"][:, 0]
    part, idx, nparts = parts_of(code)
    k = int(nparts[part][0])
    assert len(split["tasks"]) == len(whole["tasks"]) + (k - 1) * 2 * (t - 1)


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
    part, idx, _ = parts_of(code)
    trsms = np.where((kind == TRSMS) & (idx == 0))[0]
    assert len(trsms) == 2 * t * s and np.all(part[trsms])
    pr = preds_of(p)
    for v in trsms:
        ups = [u for u in pr[v] if kind[u] == GEMMS and tasks[u, 1] == tasks[v, 1]]
        assert all(part[u] for u in ups)
    n_later = int((part & (idx != 0)).sum())
    whole = spd.plan_export(t, workers=8, steps=steps, rhs_tiles=s, no_split=1)
    assert len(tasks) == len(whole["tasks"]) + n_later


def test_workspace_task_bound_covers_every_plan():
    """The device workspace sizes its per-task arrays with a bound on the
    number of tasks (paper tasks, barriers, the solve's, and the further row
    parts); every plan the FP64 form can run must fit it."""
    def bound(t, s):
        return (3 * (t * (t - 1) * (t - 2) // 6) + 6 * (t * (t - 1) // 2) + 3 * t + 2
                + 2 * t * t * s + 3 * (2 * t + 4 * t * s))
    for t in [1, 2, 3, 4, 5, 8, 13, 20]:
        for steps, s in [(7, 0), (1, 0), (6, 0), (9, 1), (9, 3), (8, 1), (8, 2)]:
            for chain in (1, 8):
                for opts in (dict(), dict(renamed=0), dict(pipelined=0)):
                    p = spd.plan_export(t, workers=256, steps=steps, rhs_tiles=s, chain=chain,
                                        **opts)
                    assert len(p["tasks"]) <= bound(t, s), (t, steps, s, chain, opts)
