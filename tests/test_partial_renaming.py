"""Memory-constrained partial renaming (Section 3, "Array renaming"; the
conclusion's question of performance under a memory constraint), on the CPU.

With opts.rename_tiles = k only whole tile rows of the copies B (of L) and C
(of L^{-1}) are renamed, at most k copy tiles, chosen greedily by the
critical path they shorten; the other rows are read in place, with the
paper's anti-dependences.  Pins:
  * the end points: a budget too small for any row gives the in-place DAG's
    critical path, a budget of 2T the renamed DAG's (Table 1);
  * the critical path never grows with the budget;
  * the plan touches at most T + (copy tiles) + 2t pool tiles;
  * every plan, executed by the host tile executor in random topological
    orders, gives the same bits in every order and the oracle's inverse."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
import tile_executor as tx
from paper_1002_4057_amd import inputs


def _cp(t, **opts):
    return spd.plan_stats(t, **opts)["cp_plan"]


@pytest.mark.parametrize("t", [3, 4, 6, 8])
def test_end_points_are_the_in_place_and_renamed_dags(t):
    T = t * (t + 1) // 2
    in_place = _cp(t, renamed=0)
    renamed = _cp(t)
    assert renamed == 5 * t - 2          # Table 1, pipelined
    assert _cp(t, rename_tiles=2 * T) == renamed
    # one tile: only row 0 of B or C fits, which the in-place DAG does not need
    assert _cp(t, rename_tiles=1) <= in_place
    assert _cp(t, rename_tiles=1) > renamed


@pytest.mark.parametrize("t", [4, 6, 8, 12])
def test_critical_path_does_not_grow_with_the_budget(t):
    T = t * (t + 1) // 2
    cps = [_cp(t, rename_tiles=k) for k in range(1, 2 * T + 1, max(1, T // 8))]
    cps.append(_cp(t))
    assert all(a >= b for a, b in zip(cps, cps[1:])), cps
    assert cps[0] > cps[-1]


@pytest.mark.parametrize("t", [8, 16, 24, 33, 64])
def test_half_of_the_copies_reach_the_renamed_critical_path(t):
    """T copy tiles, half of full renaming, already give the renamed DAG's
    critical path 5t - 2 (the rows chosen: the last C row and the B rows but
    the last, T tiles): the anti-dependences that step 3 keeps by reading
    the other rows in place stay off the critical path of the pipelined
    DAG."""
    T = t * (t + 1) // 2
    assert _cp(t, rename_tiles=T) == 5 * t - 2
    assert _cp(t, rename_tiles=T // 2) > 5 * t - 2


def _max_tile(plan):
    tk = plan["tasks"]
    m = int(max(tk[:, 1].max(), tk[:, 2].max(), tk[:, 3].max(), tk[:, 4].max()))
    pot = (tk[:, 0] & 0xFF) == tx.POTRF
    if pot.any():
        m = max(m, int(tk[pot, 5].max()) + plan["t"])   # D_j^T = D_j + t
    return m


@pytest.mark.parametrize("t,k", [(6, 5), (6, 12), (6, 30), (8, 20), (8, 50)])
def test_pool_shrinks_to_the_budget(t, k):
    T = t * (t + 1) // 2
    plan = spd.plan_export(t, workers=4, rename_tiles=k)
    assert _max_tile(plan) < T + k + 2 * t
    full = spd.plan_export(t, workers=4)
    assert _max_tile(full) >= 3 * T


@pytest.mark.parametrize("k", [1, 4, 9, 15, 27])
def test_partial_plans_execute_to_the_inverse_in_any_order(k):
    nb, n = 4, 23                        # t = 6, ragged last tile
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=31).numpy()
    ref = oracle.spd_inverse(a)
    plan = spd.plan_export(t, workers=5, rename_tiles=k)
    rng = np.random.default_rng(k)
    first = None
    for _ in range(4):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        x = tx.execute(plan, a, nb, order)
        if first is None:
            first = x
            assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-12
        else:
            assert np.array_equal(x, first)


def test_rename_budget_is_ignored_outside_the_inverse():
    # the Cholesky factor alone has no renaming copies to save
    a = spd.plan_export(5, steps=1, workers=3, rename_tiles=3)
    b = spd.plan_export(5, steps=1, workers=3)
    assert np.array_equal(a["tasks"], b["tasks"])
