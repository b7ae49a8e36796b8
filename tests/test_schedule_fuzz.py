"""Schedule fuzzing of the planner's DAG on the CPU (the race detector).

The plan the device runs is executed on the host with numpy tile operations
(tests/tile_executor.py) in many random topological orders.  Because every
tile's updates are totally ordered by the hazard edges, each order must give
a result bit-identical to program order; and dropping a single
write-after-read edge of the in-place variant must let some order read a
tile after it was overwritten, changing the result.  The program-order result
is also checked against the oracle."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs
import tile_executor as tx

VARIANTS = [
    dict(renamed=1, loop_order=0, pipelined=1),
    dict(renamed=1, loop_order=0, pipelined=0),
    dict(renamed=1, loop_order=1, pipelined=1),
    dict(renamed=0, loop_order=0, pipelined=1),
    dict(renamed=0, loop_order=0, pipelined=1, trtri_first=1),
    dict(renamed=1, loop_order=0, pipelined=1, trtri_first=1),
    dict(renamed=1, loop_order=0, pipelined=1, parts=2),
    dict(renamed=1, loop_order=0, pipelined=1, parts=4),
]


@pytest.mark.parametrize("opts", VARIANTS, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()))
def test_random_orders_bit_identical_and_match_oracle(opts):
    nb, n = 4, 21                       # t = 6, ragged last tile
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=3).numpy()
    plan = spd.plan_export(t, workers=5, **opts)
    ref = tx.execute(plan, a, nb)
    rel = np.linalg.norm(ref - oracle.spd_inverse(a)) / np.linalg.norm(ref)
    assert rel < 1e-13
    rng = np.random.default_rng(0)
    for _ in range(12):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        np.testing.assert_array_equal(tx.execute(plan, a, nb, order), ref)
    # the device dispatch order too
    np.testing.assert_array_equal(tx.execute(plan, a, nb, plan["order"]), ref)


def _war_edges(plan):
    """Edges u -> v where v overwrites a tile that u really reads (and u does
    not write), i.e. anti-dependences the executor relies on."""
    tasks, succ = plan["tasks"], plan["succ"]
    out = []
    for u in range(len(tasks)):
        ku, ou, au, bu = (int(x) for x in tasks[u, :4])
        reads = {x for x in (au, bu) if x >= 0}
        if (ku & 0xFF) in tx.PRODUCTS and (ku >> 8) & tx.F_ACC:
            reads.add(ou)
        writes_u = {ou, int(tasks[u, 4]), int(tasks[u, 5])}
        for v in succ[tasks[u, 6]:tasks[u, 7]]:
            v = int(v)
            wv = {int(tasks[v, 1]), int(tasks[v, 4]), int(tasks[v, 5])} - {-1}
            if (reads - writes_u) & wv:
                out.append((u, v))
    return out


def _reachable_without(tasks, succ, src, dst, skip):
    stack, seen = [src], {src}
    while stack:
        x = stack.pop()
        for s in succ[tasks[x, 6]:tasks[x, 7]]:
            s = int(s)
            if (x, s) == skip or s in seen:
                continue
            if s == dst:
                return True
            seen.add(s)
            stack.append(s)
    return False


def test_dropping_a_war_edge_breaks_the_in_place_variant():
    nb, n = 3, 12
    t = n // nb
    a = inputs.wishart_shift(n, seed=4).numpy()
    plan = spd.plan_export(t, workers=3, renamed=0, trtri_first=1)
    ref = tx.execute(plan, a, nb)
    tasks, succ = plan["tasks"], plan["succ"]
    broken = 0
    candidates = [e for e in _war_edges(plan) if not _reachable_without(tasks, succ, e[0], e[1], e)]
    assert candidates, "the in-place plan must contain essential anti-dependences"
    rng = np.random.default_rng(1)
    for (u, v) in candidates[:6]:
        # an order of the weakened DAG that runs the writer before the reader
        for _ in range(200):
            order = tx.random_topological_order(tasks, succ, rng, removed={(u, v)})
            pos = {x: i for i, x in enumerate(order)}
            if pos[v] < pos[u]:
                break
        else:
            continue
        if not np.array_equal(tx.execute(plan, a, nb, order), ref):
            broken += 1
    assert broken >= 1


def test_renamed_variant_has_no_step3_anti_dependences_on_inputs():
    # with renaming, step 3 reads only the copy C, so none of its reads is a
    # tile that a later task overwrites
    plan = spd.plan_export(5, renamed=1)
    wars = [e for e in _war_edges(plan) if plan["step"][e[0]] == 3]
    assert wars == []
