"""Chained device tasks (CPU only: the planner is host code in the library).

With chain > 1 the planner contracts consecutive products of one output
tile into one device task.  The contraction must not change what is
computed: expanding every chained task into its links gives, tile by tile,
the same sequence of products (operands, flags, order) as the plan with one
device task per task of the paper's stream, and the statistics (Table 1)
still describe the paper's DAG.  The contracted DAG must stay acyclic with
program order topological, never hold a product's intermediate result that
another task reads, and leave the last product before a chain's closing task
on its own.  (The schedule-fuzz tests run contracted plans in random
topological orders.)"""
import numpy as np
import pytest

import paper_1002_4057_amd as spd

NOP, SYRK1, POTRF, GEMM1, TRSM1, TRTRI = 0, 1, 2, 3, 4, 5
F_TA, F_TB, F_MA, F_MB, F_LOWER, F_NEG, F_ACC, F_COPYT = 1, 2, 4, 8, 16, 32, 64, 128
LINKS_SHIFT, LINK_KLAST, K_KLAST = 20, 1 << 30, 1 << 19
NC_A, NC_B = 1 << 17, 1 << 18
VARIANTS = [dict(), dict(pipelined=0), dict(renamed=0), dict(trtri_first=1), dict(loop_order=1),
            dict(renamed=0, trtri_first=1)]


def nlinks(code):
    return (int(code) >> LINKS_SHIFT) & 0xF


def expand(p):
    """Program-order list of (out, a, b, flags, last-block mark, copy) per
    product link, plus
    the non-product tasks as (kind, out) markers.  (The L2-cacheable read
    marks are left out: chained tasks read device-coherent.)"""
    seq = []
    for task in p["tasks"]:
        code, out, a, b, cp, aux = (int(x) for x in task[:6])
        kind, f = code & 0xFF, (code >> 8) & 0xFF
        if kind in (NOP, POTRF, TRTRI):
            seq.append(("task", kind, out, cp))
            continue
        L = nlinks(code)
        ops = [(a, b, bool(code & K_KLAST))]
        for q in range(L):
            la, lb = (int(x) for x in p["links"][aux + q])
            ops.append((la & ~LINK_KLAST, lb, bool(la & LINK_KLAST)))
        for q, (oa, ob, kl) in enumerate(ops):
            fq = f if q == 0 else f | F_ACC
            if q < L:
                fq &= ~F_COPYT        # the copy belongs to the last link
            seq.append(("prod", out, oa, ob, fq, kl, cp if q == L else -1))
    return seq


def per_tile(seq):
    """Sequence of operations on each output tile, in program order."""
    d = {}
    for e in seq:
        out = e[2] if e[0] == "task" else e[1]
        d.setdefault(out, []).append(e)
    return d


@pytest.mark.parametrize("opts", VARIANTS)
@pytest.mark.parametrize("t", [2, 3, 5, 8, 13])
@pytest.mark.parametrize("chain", [2, 3, 8, 16])
def test_expanded_chains_match_the_paper_stream(t, chain, opts):
    base = spd.plan_export(t, workers=16, chain=1, **opts)
    ch = spd.plan_export(t, workers=16, chain=chain, **opts)
    assert len(base["links"]) == 0
    a, b = expand(base), expand(ch)
    assert len(a) == len(b)                     # same number of products and tasks
    assert per_tile(a) == per_tile(b)           # same products, same order, per tile
    n_links = sum(nlinks(c) for c in ch["tasks"][:, 0])
    assert len(ch["tasks"]) + n_links == len(base["tasks"])
    assert len(ch["links"]) == n_links


@pytest.mark.parametrize("opts", VARIANTS)
@pytest.mark.parametrize("t", [4, 9, 16])
def test_statistics_describe_the_paper_dag(t, opts):
    assert spd.plan_stats(t, chain=1, **opts) == spd.plan_stats(t, chain=8, **opts)
    assert spd.plan_stats(t, chain=1, **opts) == spd.plan_stats(t, chain=16, **opts)


@pytest.mark.parametrize("opts", VARIANTS)
@pytest.mark.parametrize("t", [3, 7, 12])
def test_contracted_dag_structure(t, opts):
    p = spd.plan_export(t, workers=32, chain=8, **opts)
    tasks, succ, order = p["tasks"], p["succ"], p["order"]
    n = len(tasks)
    # program order is topological, and the dispatch order is a permutation
    for v in range(n):
        for s in succ[tasks[v, 6]:tasks[v, 7]]:
            assert s > v
    assert sorted(order.tolist()) == list(range(n))
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    for v in range(n):
        for s in succ[tasks[v, 6]:tasks[v, 7]]:
            assert pos[s] > pos[v]            # dispatch order is topological too
    for v in range(n):
        code = int(tasks[v, 0])
        L = nlinks(code)
        if not L:
            continue
        f = (code >> 8) & 0xFF
        # a chain reads both operands along columns and never reads its output
        assert f & F_TB and not f & (F_TA | F_MA | F_MB)
        for q in range(L):
            la, lb = (int(x) for x in p["links"][tasks[v, 5] + q])
            la &= ~LINK_KLAST
            assert la != tasks[v, 1] and lb != tasks[v, 1]
        assert not code & (NC_A | NC_B)       # chained tasks read device-coherent


@pytest.mark.parametrize("t", [4, 8, 16])
def test_last_product_before_closing_task_runs_alone(t):
    """In the paper's stream, the product right before a tile's closing task
    (POTRF, TRSM, or the end of the plan) waits for the most recently
    finished operand: it must never be folded into an earlier task."""
    base = spd.plan_export(t, workers=16, chain=1)
    ch = spd.plan_export(t, workers=16, chain=8)
    # the products of the chained plan that carry links: their final link
    # must be followed (on the same tile) by another chainable product
    seq = per_tile(expand(ch))
    chained_last = set()
    k = 0
    for task in ch["tasks"]:
        L = nlinks(task[0])
        if L:
            chained_last.add((int(task[1]), k + L))   # (tile, index of last link on it)
        k += 1 + L
    # index products per tile in the expanded sequence
    flat = expand(ch)
    tile_pos = {}
    for i, e in enumerate(flat):
        out = e[2] if e[0] == "task" else e[1]
        tile_pos.setdefault(out, []).append(i)
    for out, last in chained_last:
        lst = tile_pos[out]
        j = lst.index(last)
        assert j + 1 < len(lst), "a chain ends the tile's stream"
        nxt = flat[lst[j + 1]]
        assert nxt[0] == "prod" and nxt[4] & F_ACC and nxt[2] != out and nxt[3] != out
    assert seq  # non-empty
    assert len(ch["tasks"]) <= len(base["tasks"])


@pytest.mark.parametrize("t,workers", [(16, 16), (32, 64), (64, 256)])
def test_chains_form_where_operands_are_ready_early(t, workers):
    """Links join a chain only when the simulated schedule has their operands
    ready (give or take the slack) by the time the chain reaches them; at
    realistic sizes most of the step-3 products (operands made in earlier
    steps) still chain."""
    base = spd.plan_export(t, workers=workers, chain=1)
    ch = spd.plan_export(t, workers=workers, chain=8)
    assert len(ch["tasks"]) < 0.55 * len(base["tasks"])
    step3 = ch["step"] == 3
    nl = (ch["tasks"][:, 0] >> LINKS_SHIFT) & 0xF
    assert nl[step3].sum() > 0.5 * step3.sum()


@pytest.mark.parametrize("bad", [dict(chain=17), dict(chain=-1), dict(per_cu=3), dict(per_cu=-1)])
def test_chain_and_per_cu_options_range_checked(bad):
    import ctypes
    from paper_1002_4057_amd import _lib
    lib = spd._lib.load()
    o = _lib.make_opts(**bad)
    assert lib.spd_inverse(4, ctypes.c_void_p(8), 4, 0, None, 0, None, ctypes.byref(o), None,
                           None) < 0


# reduction index of each product kind in the paper's (i, j, k) naming
KBLOCK = {1: "k", 3: "k", 4: "j", 6: "i", 7: "k", 8: "j", 9: "i", 10: "i", 11: "k", 12: "k"}


@pytest.mark.parametrize("opts", [dict(), dict(pipelined=0), dict(trtri_first=1),
                                  dict(loop_order=1), dict(renamed=0)])
@pytest.mark.parametrize("t", [1, 2, 3, 4, 6])
def test_last_block_reduction_marks(t, opts):
    """K_KLAST is set exactly on the column-form products whose reduction
    index (k for GEMM and SYRK, j for the TRSMs, i for the TRMMs and LAUUM)
    is the last tile block; the device then skips the padded k-panels."""
    p = spd.plan_export(t, workers=4, chain=1, **opts)
    for task, packed in zip(p["tasks"], p["idx"]):
        code = int(task[0])
        kind, f = code & 0xFF, (code >> 8) & 0xFF
        if kind not in KBLOCK:
            assert not code & K_KLAST
            continue
        ijk = {"i": (int(packed) >> 20) & 1023, "j": (int(packed) >> 10) & 1023,
               "k": int(packed) & 1023}
        column = f & F_TB and not f & (F_TA | F_MA | F_MB)
        expect = bool(column) and ijk[KBLOCK[kind]] == t - 1
        assert bool(code & K_KLAST) == expect, (kind, ijk)
