"""The steps of Algorithm 1 on their own (CPU only: planner and host checks).

spd_cholesky runs the plan of step 1 alone and spd_inverse_from_factor the
plan of steps 2 and 3 after a prologue that makes what step 1 leaves for
step 2 (the transposed renaming copies of L's tiles and the inverted
diagonal tiles).  Here the exported partial plans are executed by the host
tile executor in program order and in random topological orders, and
checked against the oracle: the factor against its Cholesky step, the
inverse from the oracle's factor against its full inverse."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
from paper_1002_4057_amd import _lib, inputs
import tile_executor as tx

VARIANTS = [dict(), dict(renamed=0), dict(pipelined=0), dict(chain=1), dict(loop_order=1),
            dict(trtri_first=1)]


def lower_from_pool(pool, t, nb, n):
    m = t * nb
    full = np.zeros((m, m))
    for i in range(t):
        for j in range(i + 1):
            full[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = pool[tx.tri(i, j)]
    return np.tril(full)[:n, :n]


def run(plan, pool, order=None):
    tasks = plan["tasks"]
    for v in (range(len(tasks)) if order is None else order):
        tx.run_task(pool, tasks[v], plan["t"], plan.get("links"))
    return pool


def factor_prologue(pool, t):
    """What step 1 leaves for step 2, from the factor's tiles: B_ij = L_ij^T
    (i > j), D_j = L_jj^{-1} and D_j^T."""
    T = t * (t + 1) // 2
    for i in range(t):
        for j in range(i):
            pool[T + tx.tri(i, j)] = pool[tx.tri(i, j)].T
        x = np.tril(np.linalg.inv(np.tril(pool[tx.tri(i, i)])))
        pool[3 * T + i] = x
        pool[3 * T + t + i] = x.T
    return pool


@pytest.mark.parametrize("opts", VARIANTS, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()) or "default")
def test_cholesky_plan_gives_the_factor_in_any_order(opts):
    nb, n = 4, 21                        # t = 6, ragged last tile
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=4).numpy()
    plan = spd.plan_export(t, workers=5, steps=1, **opts)
    assert set(plan["step"].tolist()) <= {0, 1}
    ref = lower_from_pool(run(plan, tx.to_pool(a, t, nb)), t, nb, n)
    lo = oracle.potrf(a)
    assert np.linalg.norm(ref - lo) / np.linalg.norm(lo) < 1e-13
    rng = np.random.default_rng(1)
    for _ in range(8):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        got = lower_from_pool(run(plan, tx.to_pool(a, t, nb), order), t, nb, n)
        np.testing.assert_array_equal(got, ref)


def test_cholesky_plan_stores_every_factor_tile_and_no_unread_copy():
    """Step 1 alone: each diagonal factor tile is a final value (the copy-out
    reads it), so no POTRF drops its factor; the renaming copies B = L^T
    that only step 2 reads are not stored."""
    plan = spd.plan_export(7, workers=4, steps=1)
    kinds = plan["tasks"][:, 0]
    potrf = (kinds & 0xFF) == tx.POTRF
    assert potrf.sum() == 7
    assert not (kinds[potrf] & tx.POTRF_FACTOR_DEAD).any()
    assert (plan["tasks"][:, 4] == -1).all()
    full = spd.plan_export(7, workers=4)
    fk = full["tasks"][:, 0]
    assert (fk[(fk & 0xFF) == tx.POTRF] & tx.POTRF_FACTOR_DEAD).all()


INVT_DEAD = 1 << 29


@pytest.mark.parametrize("opts", [dict(), dict(renamed=0, trtri_first=1), dict(chain=1)])
def test_transposed_inverse_stored_only_where_read(opts):
    """POTRF(j) stores D_j and D_j^T; no task of the factor alone reads D_j^T
    (its TRSMs multiply by D_j), so there the planner marks every POTRF to
    skip it, and in the inverse and the solve (TRSM2R, TRTRI's copy into
    C_jj, the backward substitution read D_j^T) it marks none.  Checked
    against the operands of the plan itself: D_j^T is tile d_base + t + j."""
    t = 7
    for steps, s in ((1, 0), (7, 0), (9, 2)):
        plan = spd.plan_export(t, workers=4, steps=steps, rhs_tiles=s, **opts)
        tk = plan["tasks"]
        kinds = tk[:, 0]
        potrf = np.where((kinds & 0xFF) == tx.POTRF)[0]
        assert len(potrf) == t
        read = set(tk[:, 2].tolist()) | set(tk[:, 3].tolist())
        read |= set((plan["links"][:, 0] & ~(1 << 30)).tolist()) | set(plan["links"][:, 1].tolist())
        for v in potrf:
            dt = int(tk[v, 5]) + t          # aux = D_j, D_j^T follows the t tiles of D
            assert bool(kinds[v] & INVT_DEAD) == (dt not in read), (steps, v)
        assert (kinds[potrf] & INVT_DEAD).all() == (steps == 1)


@pytest.mark.parametrize("opts", VARIANTS, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()) or "default")
def test_inverse_from_factor_plan_in_any_order(opts):
    nb, n = 4, 21
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=5).numpy()
    lo = oracle.potrf(a)
    plan = spd.plan_export(t, workers=5, steps=6, **opts)
    assert set(plan["step"].tolist()) <= {0, 2, 3}
    assert not ((plan["tasks"][:, 0] & 0xFF) == tx.POTRF).any()
    ref = tx.from_pool(run(plan, factor_prologue(tx.to_pool(lo, t, nb), t)), t, nb, n)
    x = oracle.spd_inverse(a)
    assert np.linalg.norm(ref - x) / np.linalg.norm(x) < 1e-12
    rng = np.random.default_rng(2)
    for _ in range(8):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        got = tx.from_pool(run(plan, factor_prologue(tx.to_pool(lo, t, nb), t), order), t, nb, n)
        np.testing.assert_array_equal(got, ref)


def test_partial_plans_have_the_paper_task_counts():
    """Step 1: t POTRF, t(t-1)/2 SYRK and TRSM, (t-1)t(t-2)/6 GEMM; steps 2
    and 3: t TRTRI, no POTRF; the three together are the full plan."""
    t = 9
    c = lambda p, k: int(((p["tasks"][:, 0] & 0xFF) == k).sum())  # noqa: E731
    p1 = spd.plan_export(t, steps=1, chain=1)
    p6 = spd.plan_export(t, steps=6, chain=1)
    p7 = spd.plan_export(t, steps=7, chain=1)
    assert c(p1, tx.POTRF) == t and c(p1, tx.SYRK1) == t * (t - 1) // 2
    assert c(p1, tx.TRSM1) == t * (t - 1) // 2 and c(p1, tx.GEMM1) == (t - 1) * t * (t - 2) // 6
    assert c(p6, tx.TRTRI) == t and c(p6, tx.POTRF) == 0
    assert len(p1["tasks"]) + len(p6["tasks"]) == len(p7["tasks"])


def test_invalid_steps_rejected():
    with pytest.raises(ValueError):
        spd.plan_export(4, steps=3)


@pytest.mark.parametrize("name", ["spd_cholesky", "spd_inverse_from_factor"])
@pytest.mark.parametrize("args,code", [
    ((-1, 8, 1), -1),      # n < 0
    ((4, None, 4), -2),    # null matrix
    ((4, 8, 3), -3),       # lda < n
    ((4, 8, 4), -4),       # null workspace
])
def test_step_entry_points_reject_invalid_arguments_on_host(name, args, code):
    lib = _lib.load()
    n, a, lda = args
    o = _lib.make_opts()
    fn = getattr(lib, name)
    assert fn(n, a and ctypes.c_void_p(a), lda, None, 0, None, ctypes.byref(o), None, None) == code


@pytest.mark.parametrize("name", ["spd_cholesky", "spd_inverse_from_factor"])
def test_step_entry_points_reject_bad_options(name):
    lib = _lib.load()
    o = _lib.make_opts(chain=40)
    assert getattr(lib, name)(4, ctypes.c_void_p(8), 4, ctypes.c_void_p(8), 1 << 20, None,
                              ctypes.byref(o), None, None) == -7


def rhs_pool(pool, b, t, nb):
    """The pool with right-hand-side tiles appended: R_ic^T at 3T + 2t + i + t c."""
    n, nrhs = b.shape
    s = -(-nrhs // nb)
    full = np.zeros((t * nb, s * nb))
    full[:n, :nrhs] = b
    tiles = [full[i * nb:(i + 1) * nb, c * nb:(c + 1) * nb].T for c in range(s) for i in range(t)]
    return np.concatenate([pool, np.array(tiles)]), s


def rhs_from_pool(pool, t, nb, n, nrhs, s):
    base = len(pool) - t * s
    full = np.zeros((t * nb, s * nb))
    for c in range(s):
        for i in range(t):
            full[i * nb:(i + 1) * nb, c * nb:(c + 1) * nb] = pool[base + i + t * c].T
    return full[:n, :nrhs]


@pytest.mark.parametrize("opts", VARIANTS, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()) or "default")
def test_solve_plan_factor_and_substitutions_in_any_order(opts):
    """steps = 9: step 1 and the forward and backward substitutions in one
    DAG; the factor in A and X in the right-hand-side tiles, in any
    topological order, against the oracle's factor and solve."""
    nb, n, nrhs = 4, 21, 6                 # t = 6, s = 2 (ragged in both)
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=6).numpy()
    b = np.random.default_rng(6).standard_normal((n, nrhs))
    pool0, s = rhs_pool(tx.to_pool(a, t, nb), b, t, nb)
    plan = spd.plan_export(t, workers=5, steps=9, rhs_tiles=s, **opts)
    assert set(plan["step"].tolist()) <= {0, 1, 4}
    ref_pool = run(plan, pool0.copy())
    x = rhs_from_pool(ref_pool, t, nb, n, nrhs, s)
    lo = oracle.potrf(a)
    xo = oracle.potrs(lo, b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-12
    assert np.linalg.norm(lower_from_pool(ref_pool, t, nb, n) - lo) / np.linalg.norm(lo) < 1e-13
    rng = np.random.default_rng(7)
    for _ in range(6):
        order = tx.random_topological_order(plan["tasks"], plan["succ"], rng)
        np.testing.assert_array_equal(run(plan, pool0.copy(), order), ref_pool)


@pytest.mark.parametrize("opts", [dict(), dict(renamed=0)], ids=["renamed", "in-place"])
def test_solve_plan_with_a_given_factor(opts):
    """steps = 8: the substitutions alone, after the factor prologue."""
    nb, n, nrhs = 4, 18, 3
    t = -(-n // nb)
    a = inputs.wishart_shift(n, seed=8).numpy()
    b = np.random.default_rng(8).standard_normal((n, nrhs))
    lo = oracle.potrf(a)
    pool0, s = rhs_pool(factor_prologue(tx.to_pool(lo, t, nb), t), b, t, nb)
    plan = spd.plan_export(t, workers=3, steps=8, rhs_tiles=s, **opts)
    assert set(plan["step"].tolist()) <= {4}
    x = rhs_from_pool(run(plan, pool0.copy()), t, nb, n, nrhs, s)
    xo = oracle.potrs(lo, b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-12


def test_solve_plan_task_counts_and_invalid_combinations():
    t, s = 7, 3
    p9 = spd.plan_export(t, steps=9, rhs_tiles=s, chain=1)
    p1 = spd.plan_export(t, steps=1, chain=1)
    k = p9["tasks"][:, 0] & 0xFF
    # forward and backward: per right-hand-side tile column, t(t-1)/2 updates
    # and t multiplications by a diagonal inverse each
    assert int((k == tx.GEMMS).sum()) == 2 * s * t * (t - 1) // 2
    assert int((k == tx.TRSMS).sum()) == 2 * s * t
    assert len(p9["tasks"]) == len(p1["tasks"]) + 2 * s * (t * (t - 1) // 2 + t)
    for steps, rhs in ((9, 0), (8, 0), (7, 1), (9, 65), (5, 0)):
        with pytest.raises(ValueError):
            spd.plan_export(4, steps=steps, rhs_tiles=rhs)


@pytest.mark.parametrize("name", ["spd_solve", "spd_solve_from_factor"])
@pytest.mark.parametrize("args,code", [
    ((-1, 1, 8, 1, 8, 1), -1),       # n < 0
    ((4, -1, 8, 4, 8, 4), -2),       # nrhs < 0
    ((4, 8193, 8, 4, 8, 4), -2),     # nrhs too large
    ((4, 1, None, 4, 8, 4), -3),     # null matrix
    ((4, 1, 8, 3, 8, 4), -4),        # lda < n
    ((4, 1, 8, 4, None, 4), -5),     # null right-hand sides
    ((4, 1, 8, 4, 8, 3), -6),        # ldb < n
    ((4, 1, 8, 4, 8, 4), -7),        # null workspace
])
def test_solve_entry_points_reject_invalid_arguments_on_host(name, args, code):
    lib = _lib.load()
    n, nrhs, a, lda, b, ldb = args
    o = _lib.make_opts()
    fn = getattr(lib, name)
    assert fn(n, nrhs, a and ctypes.c_void_p(a), lda, b and ctypes.c_void_p(b), ldb, None, 0, None,
              ctypes.byref(o), None, None) == code


@pytest.mark.parametrize("name", ["spd_cholesky", "spd_inverse_from_factor"])
@pytest.mark.parametrize("opts", [dict(renamed=0), dict(rename_tiles=5)])
def test_step_entry_points_run_the_renamed_plan_only(name, opts):
    """The steps on their own use the standard layout of the renamed plan
    (the factor prologue writes every copy): the in-place and partially
    renamed options, whose workspace query is smaller, are rejected."""
    lib = _lib.load()
    o = _lib.make_opts(**opts)
    assert getattr(lib, name)(4, ctypes.c_void_p(8), 4, ctypes.c_void_p(8), 1 << 20, None,
                              ctypes.byref(o), None, None) == -7
    b = ctypes.c_void_p(8)
    assert lib.spd_solve(4, 1, ctypes.c_void_p(8), 4, b, 4, ctypes.c_void_p(8), 1 << 20, None,
                         ctypes.byref(o), None, None) == -10
