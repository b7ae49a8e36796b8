"""The batched form's task lists and dispatch order, on the CPU (no GPU).

The device runs one dependency-tracked DAG over the whole batch: each matrix
its template (copy-in, the plan of Algorithm 1 for its tile count, copy-out,
or one small-matrix task), tickets in the dispatch order the host builds.
These tests check that the dispatch order is a permutation of every
(matrix, task) and topological, which makes the device loop deadlock-free
for any number of workers, and they execute the tickets in that order with
the host tile executor: every matrix above one tile must come out as the
oracle's inverse."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
import tile_executor as tx
from paper_1002_4057_amd import inputs

NB = 128
BCOPYIN, BCOPYOUT, BSMALL = 16, 17, 18
BM_PREV = 1 << 8    # the matrix's pool slot had an earlier occupant
ORDERS = [50, 129, 300, 512, 20, 256, 140, 0, 385, 128, 700]


def _templates(orders, mode="fp64", **opts):
    ts = sorted({1 if n <= NB else -(-n // NB) for n in orders})
    return {t: spd.batch_template_export(t, mode, **opts) for t in ts}


def _check_order(orders, tmpl, plan):
    disp, mat = plan["disp"], plan["mat"]
    seen = {}
    for x, e in enumerate(disp.tolist()):
        m, pos = e >> 12, e & 4095
        assert (m, pos) not in seen
        seen[(m, pos)] = x
    base_of = {int(mat[m, 1]): m for m in range(len(orders))}
    for m, n in enumerate(orders):
        t = 1 if n <= NB else -(-n // NB)
        assert mat[m, 0] & 0xFF == t
        tp = tmpl[t]
        assert all((m, p) in seen for p in range(len(tp["tasks"])))
        for p, task in enumerate(tp["tasks"]):
            for s in tp["succ"][task[6]:task[7]]:
                assert seen[(m, p)] < seen[(m, int(s))], (m, p, int(s))
        # a pool slot passes from m to its next occupant after m's copy-out
        if mat[m, 3] >= 0:
            nxt = base_of[int(mat[m, 3])]
            assert mat[nxt, 0] & BM_PREV and mat[nxt, 2] == mat[m, 2]
            assert seen[(m, len(tp["tasks"]) - 1)] < seen[(nxt, 0)]
    assert len(seen) == len(disp)


def _execute(orders, mats, tmpl, plan):
    """Runs the tickets in dispatch order on host pools indexed by each
    matrix's first pool tile: a slot must be free when a copy-in task takes
    it (its previous occupant's copy-out task has run)."""
    pools, out = {}, {}
    for e in plan["disp"].tolist():
        m, pos = e >> 12, e & 4095
        n = orders[m]
        t = int(plan["mat"][m, 0]) & 0xFF
        base = int(plan["mat"][m, 2])
        task = tmpl[t]["tasks"][pos]
        kind = int(task[0]) & 0xFF
        if kind == BSMALL:
            out[m] = None                   # inverted in LDS on the device
        elif kind == BCOPYIN:
            assert base not in pools, "pool slot still in use"
            pools[base] = tx.to_pool(mats[m], t, NB)
        elif kind == BCOPYOUT:
            out[m] = tx.from_pool(pools.pop(base), t, NB, n)
        else:
            tx.run_task(pools[base], task, t, tmpl[t]["links"])
    assert not pools
    return out


@pytest.mark.parametrize("opts", [dict(batch_group=-2), dict(chain=1, batch_group=-2),
                                  dict(batch_group=1), dict(batch_group=3),
                                  dict(loop_order=1, batch_group=-2)])
@pytest.mark.parametrize("workers", [1, 5, 512])
def test_dispatch_is_topological_and_executes_to_the_inverse(opts, workers):
    mats = [inputs.wishart_shift(n, seed=60 + i, shift=0.1).numpy() if n else np.zeros((0, 0))
            for i, n in enumerate(ORDERS)]
    tmpl = _templates(ORDERS, **opts)
    plan = spd.batch_plan_export(ORDERS, workers=workers, **opts)
    _check_order(ORDERS, tmpl, plan)
    out = _execute(ORDERS, mats, tmpl, plan)
    for m, n in enumerate(ORDERS):
        if n <= NB:
            assert out[m] is None
            continue
        ref = oracle.spd_inverse(mats[m])
        ev = np.linalg.eigvalsh(mats[m])
        err = np.linalg.norm(out[m] - ref) / np.linalg.norm(ref)
        assert err <= 1e-12 * ev[-1] / ev[0], (m, n)


def test_fp32_templates_wrap_the_fp64_plan():
    """The FP32 templates are those of FP64, chained products included (the
    FP32 tile product runs chains too)."""
    tmpl = _templates([300, 700], mode="fp32")
    ref = _templates([300, 700])
    for t, tp in tmpl.items():
        kinds = tp["tasks"][:, 0] & 0xFF
        assert kinds[0] == BCOPYIN and kinds[-1] == BCOPYOUT
        assert np.array_equal(tp["tasks"], ref[t]["tasks"])
        assert np.array_equal(tp["links"], ref[t]["links"])
    plan = spd.batch_plan_export([300, 700, 90], mode="fp32", workers=64, batch_group=-2)
    _check_order([300, 700, 90], tmpl | _templates([90], mode="fp32"), plan)


def _expanded(tasks, links):
    """(out, a, b) of every tile product, chained links expanded, and the
    kinds of the other tasks."""
    prods, others = [], []
    for task in tasks:
        kind = int(task[0])
        if (kind & 0xFF) in tx.PRODUCTS:
            prods.append((int(task[1]), int(task[2]), int(task[3])))
            nl = (kind >> tx.LINKS_SHIFT) & 0xF
            for q in range(nl):
                la, lb = links[int(task[5]) + q]
                prods.append((int(task[1]), int(la) & ~tx.LINK_KLAST, int(lb)))
        else:
            others.append(kind & 0xFF)
    return sorted(prods), sorted(others)


def test_templates_wrap_the_plan_of_algorithm_1():
    """Template of t: the copy-in task, then the tile products and the other
    tasks of the plan that one worker would run (the same operand tiles; the
    template also chains each update chain's last product, as one workgroup
    runs the matrix's tasks in order), then the copy-out."""
    for t in (2, 3, 4, 16):
        tp = spd.batch_template_export(t)
        pl = spd.plan_export(t, workers=1)
        assert _expanded(tp["tasks"][1:-1], tp["links"]) == _expanded(pl["tasks"], pl["links"])
        assert len(tp["tasks"]) - 2 <= len(pl["tasks"])
        assert tp["tasks"][0, 0] == BCOPYIN and tp["tasks"][-1, 0] == BCOPYOUT
    assert len(spd.batch_template_export(16)["tasks"]) - 2 < len(spd.plan_export(16, workers=1)["tasks"])
    small = spd.batch_template_export(1)
    assert small["tasks"].shape[0] == 1 and small["tasks"][0, 0] == BSMALL


def test_pool_slots_are_recycled():
    """With the list-scheduled order, matrices that run one after another
    share pool slots: far fewer pool tiles than one pool per matrix."""
    orders = inputs.batch_orders(600, 16, 512, seed=3)
    plan = spd.batch_plan_export(orders, workers=64, batch_group=-2)
    mat = plan["mat"]
    assert (mat[:, 0] & BM_PREV).sum() > 200
    own = sum(3 * t * (t + 1) // 2 + 2 * t for t in (-(-n // NB) for n in orders) if t >= 2)
    used = max(int(mat[m, 2]) + 3 * t * (t + 1) // 2 + 2 * t
               for m, t in enumerate(int(x) & 0xFF for x in mat[:, 0]) if t >= 2)
    assert used < own / 2
    assert spd.batched_workspace_bytes(orders, workers=64, batch_group=-2) < own * 128 * 128 * 8 / 2


def test_one_workgroup_per_matrix_dispatch():
    """batch_group = -1: one ticket per matrix, the largest first; the
    workgroup runs the template in order (a topological order)."""
    orders = [100, 2048, 300, 1000, 0, 129]
    plan = spd.batch_plan_export(orders, workers=8, batch_group=-1)
    ms = (plan["disp"] >> 12).tolist()
    assert sorted(ms) == list(range(len(orders)))
    assert all(plan["disp"] & 4095 == 0)
    ts = [1 if orders[m] <= NB else -(-orders[m] // NB) for m in ms]
    assert ts == sorted(ts, reverse=True)
    for t in (2, 3, 8, 16):
        tp = spd.batch_template_export(t)
        for p, task in enumerate(tp["tasks"]):
            assert all(int(q) > p for q in tp["succ"][task[6]:task[7]])


def test_library_choice_of_schedule():
    """batch_group = 0: one workgroup per matrix when the batch has at least
    two matrices per worker, else the list-scheduled DAG."""
    many = spd.batch_plan_export([200] * 40, workers=16)
    assert len(many["disp"]) == 40                      # a ticket per matrix
    few = spd.batch_plan_export([200] * 20, workers=16)
    assert len(few["disp"]) == 20 * len(spd.batch_template_export(2)["tasks"])


def test_largest_matrices_are_dispatched_first():
    orders = [100, 2048, 300, 1000]
    plan = spd.batch_plan_export(orders, workers=4)
    first = plan["disp"][0] >> 12
    assert orders[first] == 2048


def test_invalid_arguments():
    with pytest.raises(ValueError):
        spd.batch_plan_export([2049])
    with pytest.raises(ValueError):
        spd.batch_template_export(17)
    with pytest.raises(ValueError):
        spd.batch_plan_export([100], mode="mixed_fp32")
