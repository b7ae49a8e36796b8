"""Host executor of an exported plan with numpy tile operations.

Test fixture only (never a product path): it runs the task DAG that the
device scheduler runs, one tile operation per task with the semantics of the
device kernels, in any topological order the caller chooses.  Used to check
that the planner's hazard edges make the result independent of the order
(the schedule "race detector") and to check the plan end to end against the
oracle on the CPU.
"""
import numpy as np

NOP, SYRK1, POTRF, GEMM1, TRSM1, TRTRI, TRMM2L, GEMM2, TRSM2R, TRMM3, LAUUM, GEMM3, SYRK3 = range(13)
GEMMS, TRSMS = 13, 14   # the solve with the factor
TADD = 15               # tree reduction: out (+/-)= a
POTRF_FACTOR_DEAD = 1 << 16
LINKS_SHIFT = 20   # chained products: count of further links (see plan.hpp)
PART, PART_SHIFT, PARTS4 = 1 << 24, 25, 1 << 27   # row-part task (see plan.hpp)
LINK_KLAST = 1 << 30   # link mark: reduction over the last tile block
PRODUCTS = {SYRK1, GEMM1, TRSM1, TRMM2L, GEMM2, TRSM2R, TRMM3, LAUUM, GEMM3, SYRK3, GEMMS, TRSMS}
F_TA, F_TB, F_MA, F_MB, F_LOWER, F_NEG, F_ACC, F_COPYT = 1, 2, 4, 8, 16, 32, 64, 128


def tri(i, j):
    return i * (i + 1) // 2 + j


def to_pool(a, t, nb, extra=0):
    """Lower tiles of a (zero-padded, identity on the padded diagonal), in a
    pool of the standard 3T + 2t tiles plus `extra`."""
    n = a.shape[0]
    m = t * nb
    full = np.eye(m)
    full[:n, :n] = np.tril(a)
    T = t * (t + 1) // 2
    pool = np.zeros((3 * T + 2 * t + extra, nb, nb))
    for i in range(t):
        for j in range(i + 1):
            pool[tri(i, j)] = full[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
    return pool


def from_pool(pool, t, nb, n):
    m = t * nb
    full = np.zeros((m, m))
    for i in range(t):
        for j in range(i + 1):
            full[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = pool[tri(i, j)]
    low = np.tril(full)[:n, :n]
    return low + np.tril(low, -1).T


def run_task(pool, task, t, links=None):
    """One task with the device semantics: a tile product C (+)= +-op(A) op(B)
    driven by the flags (a chained product applies its further links in
    order, each accumulating, and copies the final tile), the diagonal
    factorization, or the TRTRI copy."""
    code, out, a, b, cp, aux = (int(x) for x in task[:6])
    kind, f = code & 0xFF, (code >> 8) & 0xFF
    factor_dead = bool(code & POTRF_FACTOR_DEAD)
    if kind == NOP:
        return
    if kind in PRODUCTS and code & PART:
        # one row part of a single product: only those rows of the output
        # (and their part of the copy) are written
        nb = pool.shape[1]
        size = nb // (4 if code & PARTS4 else 2)
        idx = (code >> PART_SHIFT) & 3
        rows = slice(idx * size, (idx + 1) * size)
        A = pool[a].T if f & F_TA else pool[a]
        B = pool[b].T if f & F_TB else pool[b]
        p = (A @ B)[rows]
        if f & F_NEG:
            p = -p
        r = pool[out][rows] + p if f & F_ACC else p
        pool[out][rows] = r
        if cp >= 0:
            if f & F_COPYT:
                pool[cp][:, rows] = r.T
            else:
                pool[cp][rows] = r
    elif kind in PRODUCTS:
        ops = [(a, b)]
        for q in range((code >> LINKS_SHIFT) & 0xF):
            la, lb = (int(x) for x in links[aux + q])
            la &= ~LINK_KLAST
            ops.append((la, lb))
        for q, (oa, ob) in enumerate(ops):
            fq = f if q == 0 else f | F_ACC
            A = pool[oa].T if fq & F_TA else pool[oa]
            B = pool[ob].T if fq & F_TB else pool[ob]
            if fq & F_MA:
                A = np.triu(A) if fq & F_TA else np.tril(A)
            if fq & F_MB:
                B = np.triu(B) if fq & F_TB else np.tril(B)
            p = A @ B
            if fq & F_NEG:
                p = -p
            pool[out] = pool[out] + p if fq & F_ACC else p
        r = pool[out]
        if cp >= 0:
            pool[cp] = r.T if f & F_COPYT else r
    elif kind == POTRF:
        O = pool[out]
        L = np.linalg.cholesky(np.tril(O) + np.tril(O, -1).T)
        X = np.tril(np.linalg.inv(L))
        pool[aux] = X
        pool[aux + t] = X.T
        if not factor_dead:      # a dead factor is not stored (nothing reads it)
            pool[out] = L
            if cp >= 0:
                pool[cp] = L.T
    elif kind == TADD:
        pool[out] = pool[out] - pool[a] if f & F_NEG else pool[out] + pool[a]
    elif kind == TRTRI:
        pool[out] = pool[a]
        if cp >= 0:
            pool[cp] = pool[b]
    else:
        raise ValueError(kind)


def random_topological_order(tasks, succ, rng, removed=None):
    n = len(tasks)
    indeg = np.zeros(n, dtype=np.int64)
    for v in range(n):
        for s in succ[tasks[v, 6]:tasks[v, 7]]:
            if removed is None or (v, int(s)) not in removed:
                indeg[s] += 1
    ready = [v for v in range(n) if indeg[v] == 0]
    order = []
    while ready:
        k = int(rng.integers(len(ready)))
        v = ready.pop(k)
        order.append(v)
        for s in succ[tasks[v, 6]:tasks[v, 7]]:
            if removed is not None and (v, int(s)) in removed:
                continue
            indeg[s] -= 1
            if indeg[s] == 0:
                ready.append(int(s))
    assert len(order) == n
    return order


def execute(plan, a, nb, order=None, extra=0):
    t = plan["t"]
    pool = to_pool(a, t, nb, extra)
    tasks = plan["tasks"]
    for v in (range(len(tasks)) if order is None else order):
        run_task(pool, tasks[v], t, plan.get("links"))
    return from_pool(pool, t, nb, a.shape[0])
