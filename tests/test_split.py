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


@pytest.mark.parametrize("parts", [0, 2, 4])
@pytest.mark.parametrize("opts", [dict(), dict(chain=1), dict(renamed=0), dict(pipelined=0)])
@pytest.mark.parametrize("t", [2, 3, 6, 9])
def test_split_marks_the_step1_path(t, opts, parts):
    p = spd.plan_export(t, workers=8, parts=parts, **opts)
    tasks = p["tasks"]
    code = tasks[:, 0]
    kind = code & 0xFF
    part, idx, nparts = parts_of(code)
    heads = np.where(part & (idx == 0))[0]
    k = int(nparts[heads[0]])
    assert k in (2, 4) and np.all(nparts[part] == k)
    assert k == (parts or 4)            # library choice below 96 tiles: quarters
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


@pytest.mark.parametrize("bad", [dict(no_split=2), dict(no_split=-1), dict(parts=1),
                                 dict(parts=3), dict(parts=8), dict(parts=-2)])
def test_split_option_range_checked(bad):
    """An out-of-range no_split or parts is rejected before anything touches
    the device."""
    import ctypes
    from paper_1002_4057_amd import _lib
    lib = _lib.load()
    o = _lib.make_opts(**bad)
    assert lib.spd_inverse(4, ctypes.c_void_p(8), 4, 0, None, 0, None, ctypes.byref(o), None,
                           None) == -8


@pytest.mark.parametrize("parts", [2, 4])
def test_forced_parts_at_wide_orders(parts):
    """At 96 tiles per side and more the library picks halves; `parts` forces
    halves or quarters there too (the plan the GPU tests run at n = 16384)."""
    t = 100
    p = spd.plan_export(t, workers=512, parts=parts)
    part, idx, nparts = parts_of(p["tasks"][:, 0])
    assert np.all(nparts[part] == parts) and int(part.sum()) == parts * 2 * (t - 1)
    lib_choice = spd.plan_export(t, workers=512)
    part0, _, nparts0 = parts_of(lib_choice["tasks"][:, 0])
    assert np.all(nparts0[part0] == 2)


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


def _plan_sizes(t, workers, **opts):
    import ctypes
    from paper_1002_4057_amd import _lib
    lib = _lib.load()
    o = _lib.make_opts(**opts)
    nt, ns, nl = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    rc = lib.spdinv_plan_export_steps(7, 0, t, ctypes.byref(o), workers, None, None, None, None,
                                      None, ctypes.byref(nt), ctypes.byref(ns), None,
                                      ctypes.byref(nl))
    assert rc == 0
    return nt.value, ns.value, nl.value


def test_largest_order_plans_fit_int32_and_the_workspace_bound():
    """n = 32768 (t = 256, the largest order of the precision workload), in
    the launch the library uses there (512 workers): the default chained plan
    is exported and its int32 fields checked against the pool and the task
    count; the unchained plan with quarters (the most device tasks any FP64
    plan has at this order) must still fit the workspace's task bound."""
    t, T = 256, 256 * 257 // 2
    bound = 3 * (t * (t - 1) * (t - 2) // 6) + 6 * (t * (t - 1) // 2) + 3 * t + 2 + 3 * (2 * t)
    nt, ns, nl = _plan_sizes(t, 512, chain=1, parts=4)
    assert nt <= bound and ns < 2 ** 31
    p = spd.plan_export(t, workers=512)
    tasks, succ, links = p["tasks"], p["succ"], p["links"]
    ntask = len(tasks)
    assert ntask <= bound and len(succ) < 2 ** 31 and links.size < 2 ** 31
    pool = 3 * T + 2 * t
    assert tasks[:, 1:5].max() < pool and tasks[:, 1:5].min() >= -1
    assert np.all(tasks[:, 6] <= tasks[:, 7]) and tasks[-1, 7] == len(succ)
    assert succ.min() >= 0 and succ.max() < ntask
    assert (links[:, 0] & ~(1 << 30)).max() < pool and links[:, 1].max() < pool
    order = p["order"]
    assert np.array_equal(np.sort(order), np.arange(ntask))   # a permutation of the tasks
