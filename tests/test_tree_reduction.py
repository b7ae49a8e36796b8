"""Tree reduction of the step-2 update chains, on the CPU (no GPU).

The conclusion (Section 4) notes that the GEMM updates of a tile are
associative as well as commutative, so a tile's chain
    X_ij = -(X_ii L_ij + sum_{j<k<i} X_ik L_kj) L_jj^{-1}
may be summed as a tree instead of one sequential chain.  With
opts.tree_levels = L the planner cuts each chain into up to 2^L consecutive
ranges of k: the ranges of larger k (whose X_ik become final first) go into
partial-sum tiles Z side by side, the Z are added into A_ij in a fixed
binary tree, and the range that starts at k = j + 1 (the last X_ik to become
final) accumulates into A_ij last.  Pins:
  * an independent hazard model of step 2 (RAW, WAR and WAW over the
    paper's tiles and the partial sums, unit task weights) reproduces the
    planner's step-2 critical path, with and without the tree, in both loop
    orders and in both the renamed and the in-place form; at L = 0 it also
    reproduces Table 1's figures, which pins the model itself;
  * the UUU order, whose chains wait on their first term, gets a critical
    path about 2^L times shorter; the UDU order keeps its own (L = 1) or
    gains a constant (L = 2);
  * the counts: one tile addition per extra range, the GEMM count unchanged;
  * the plans, run by the host tile executor in random topological orders,
    give the same bits in every order (the tree is fixed, not schedule
    dependent) and the oracle's inverse; they differ from L = 0 only in
    rounding."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
import tile_executor as tx
from paper_1002_4057_amd import inputs


def _ranges(j, m, segs):
    return [(j + 1 + m * l // segs, j + 1 + m * (l + 1) // segs) for l in range(segs)]


def step2_model(t, levels, uuu, renamed):
    """Critical path (unit weights) of step 2 from the hazards of its tasks,
    written from the recurrence of Section 2 (LAPACK order: the diagonal
    tile is inverted after its column when renamed, before it in place)."""
    tasks = []     # (reads, writes)

    def op(reads, writes):
        tasks.append((reads, writes))

    zmax = (1 << levels) - 1 if levels else 0
    for j in range(t - 1, -1, -1):
        if not renamed:
            op({("A", j, j)}, {("A", j, j)})
        for i in range(t - 1, j, -1):
            op({("A", i, i), ("A", i, j)}, {("A", i, j)})
            m = i - j - 1
            lt = "A" if not renamed else "B"

            def term(k, out):
                op({("A", i, k), (lt, k, j), out}, {out})

            def seq(lo, hi, out):
                ks = range(lo, hi) if uuu else range(hi - 1, lo - 1, -1)
                for k in ks:
                    term(k, out)
            if not zmax or m < 2:
                seq(j + 1, j + 1 + m, ("A", i, j))
            else:
                segs = min(zmax + 1, m)
                rg = _ranges(j, m, segs)
                name = [("A", i, j)] + [("Z", i, j, l) for l in range(1, segs)]
                for l in range(1, segs):
                    seq(*rg[l], name[l])
                adds = {2: [(0, 1)], 3: [(1, 2), (0, 1)], 4: [(1, 2), (0, 3), (0, 1)]}[segs]
                for d, s in adds:
                    op({name[s], name[d]}, {name[d]})
                seq(*rg[0], name[0])
            djj = ("B", j, j) if renamed else ("A", j, j)
            op({djj, ("A", i, j)}, {("A", i, j)} | ({("C", i, j)} if renamed else set()))
        if renamed:
            op({("A", j, j)}, {("A", j, j), ("C", j, j)})
    last_w, readers, lp = {}, {}, []
    for reads, writes in tasks:
        preds = set()
        for r in reads:
            if r in last_w:
                preds.add(last_w[r])
        for w in writes:
            if w in last_w:
                preds.add(last_w[w])
            preds.update(readers.get(w, ()))
        v = len(lp)
        lp.append(1 + max((lp[q] for q in preds), default=0))
        for r in reads:
            readers.setdefault(r, []).append(v)
        for w in writes:
            last_w[w] = v
            readers[w] = []
    return max(lp, default=0)


@pytest.mark.parametrize("t", [2, 3, 5, 8, 13, 16, 24])
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("uuu", [0, 1])
@pytest.mark.parametrize("renamed", [1, 0])
def test_step2_critical_path_matches_the_hazard_model(t, levels, uuu, renamed):
    st = spd.plan_stats(t, renamed=renamed, loop_order=uuu, trtri_first=1 - renamed,
                        tree_levels=levels)
    assert st["cp_step"][1] == step2_model(t, levels, uuu, renamed)


def test_model_reproduces_table1_without_the_tree():
    # Table 1 (renamed: 2t - 1; in place: 3t - 3) and the UUU figures of
    # Section 3 ("Loop reversal": t^2/2 - t/2 + 2 renamed, t^2 - 2t + 3 in
    # place), for t >= 3
    for t in (3, 4, 8, 11, 16):
        assert step2_model(t, 0, 0, 1) == 2 * t - 1
        assert step2_model(t, 0, 0, 0) == 3 * t - 3
        assert step2_model(t, 0, 1, 1) == (t * t - t) // 2 + 2
        assert step2_model(t, 0, 1, 0) == t * t - 2 * t + 3


@pytest.mark.parametrize("t", [16, 32, 64])
def test_uuu_critical_path_shrinks_with_the_levels(t):
    cp = [spd.plan_stats(t, loop_order=1, tree_levels=L)["cp_step"][1] for L in (0, 1, 2)]
    assert cp[0] > 1.6 * cp[1] and cp[1] > 1.5 * cp[2]
    assert cp[0] > 2.5 * cp[2]
    udu = [spd.plan_stats(t, loop_order=0, tree_levels=L)["cp_step"][1] for L in (0, 1, 2)]
    assert udu[1] == udu[0] == 2 * t - 1
    assert udu[2] <= udu[0] + 3
    whole = [spd.plan_stats(t, loop_order=1, tree_levels=L)["cp_plan"] for L in (0, 2)]
    assert whole[1] < whole[0] / 1.8


@pytest.mark.parametrize("t", [1, 2, 3, 4, 7, 12])
@pytest.mark.parametrize("levels", [1, 2])
def test_task_counts(t, levels):
    base = spd.plan_stats(t)["count"]
    c = spd.plan_stats(t, tree_levels=levels)["count"]
    zmax = (1 << levels) - 1
    adds = sum(min(zmax + 1, i - j - 1) - 1 for i in range(t) for j in range(i) if i - j - 1 >= 2)
    assert c["TADD"] == adds
    for k in base:
        if k != "TADD":
            assert c[k] == base[k], k


def test_other_steps_are_unchanged():
    # the factor alone has no step-2 chain; step 3's chains are not reduced
    a = spd.plan_export(6, steps=1, workers=3, tree_levels=2)
    b = spd.plan_export(6, steps=1, workers=3)
    assert np.array_equal(a["tasks"], b["tasks"])
    s = spd.plan_stats(9, tree_levels=2)["cp_step"]
    assert s[0] == spd.plan_stats(9)["cp_step"][0] and s[2] == spd.plan_stats(9)["cp_step"][2]


def _run(plan, a, nb, t, order, levels):
    T = t * (t + 1) // 2
    return tx.execute(plan, a, nb, order, extra=T * ((1 << levels) - 1))


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("opts", [dict(), dict(loop_order=1), dict(renamed=0, trtri_first=1),
                                  dict(loop_order=1, chain=1), dict(rename_tiles=9)])
def test_tree_plans_execute_to_the_inverse_in_any_order(levels, opts):
    nb, n = 4, 29                        # t = 8, ragged last tile
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=44).numpy()
    ref = oracle.spd_inverse(a)
    plan = spd.plan_export(t, workers=6, tree_levels=levels, **opts)
    kinds = plan["tasks"][:, 0] & 0xFF
    assert (kinds == tx.TADD).sum() > 0
    rng = np.random.default_rng(levels)
    first = None
    for _ in range(4):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        x = _run(plan, a, nb, t, order, levels)
        if first is None:
            first = x
            assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-12
        else:
            assert np.array_equal(x, first)
    # the same plan for another worker count (other chains) gives the same bits
    other = spd.plan_export(t, workers=1, tree_levels=levels, **opts)
    assert np.array_equal(_run(other, a, nb, t, None, levels), first)


@pytest.mark.parametrize("levels", [1, 2])
def test_from_factor_plans_use_the_tree(levels):
    """steps = 6 (X^T X from a given factor): the partial sums sit after the
    standard layout's D and D^T."""
    from test_steps import factor_prologue, run
    nb, n = 4, 26
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=45).numpy()
    lo = oracle.potrf(a)
    plan = spd.plan_export(t, steps=6, workers=3, tree_levels=levels)
    assert ((plan["tasks"][:, 0] & 0xFF) == tx.TADD).any()
    T = t * (t + 1) // 2
    x = oracle.spd_inverse(a)
    rng = np.random.default_rng(7)
    first = None
    for _ in range(3):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        pool = factor_prologue(tx.to_pool(lo, t, nb, extra=T * ((1 << levels) - 1)), t)
        got = tx.from_pool(run(plan, pool, order), t, nb, n)
        if first is None:
            first = got
            assert np.linalg.norm(got - x) / np.linalg.norm(x) < 1e-12
        else:
            assert np.array_equal(got, first)


@pytest.mark.parametrize("levels", [-1, 3])
def test_invalid_levels_are_rejected_on_host(levels):
    import ctypes
    from paper_1002_4057_amd import _lib
    lib = _lib.load()
    o = _lib.make_opts(tree_levels=levels)
    assert lib.spd_inverse_from_factor(4, ctypes.c_void_p(8), 4, ctypes.c_void_p(8), 1 << 20, None,
                                       ctypes.byref(o), None, None) == -7


@pytest.mark.parametrize("t", [3, 8, 24, 40])
@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("opts", [dict(chain=1), dict(chain=1, parts=4), dict(), dict(renamed=0)])
def test_workspace_holds_a_counter_for_every_task(t, levels, opts):
    """The workspace holds the pool (with the partial sums) and one in-degree
    counter per device task: one task per product (chain = 1) gives the most
    tasks, and the tile additions come on top of the paper's tasks."""
    n = t * 128 - 5
    T = t * (t + 1) // 2
    plan = spd.plan_export(t, workers=37, tree_levels=levels, **opts)
    pool_tiles = (T if opts.get("renamed", 1) == 0 else 3 * T) + 2 * t + T * ((1 << levels) - 1)
    ws = spd.workspace_bytes(n, tree_levels=levels, **opts)
    assert ws - pool_tiles * 128 * 128 * 8 - 256 >= 4 * len(plan["tasks"])
