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


def tri(i, j):
    return i * (i + 1) // 2 + j


def to_pool(a, t, nb):
    """Lower tiles of a (zero-padded, identity on the padded diagonal)."""
    n = a.shape[0]
    m = t * nb
    full = np.eye(m)
    full[:n, :n] = np.tril(a)
    T = t * (t + 1) // 2
    pool = np.zeros((3 * T + t, nb, nb))
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


def run_task(pool, task):
    kind, out, a, b, cp, aux = (int(x) for x in task[:6])
    if kind == NOP:
        return
    O = pool[out]
    A = pool[a] if a >= 0 else None
    B = pool[b] if b >= 0 else None
    if kind == SYRK1:
        r = O - A @ A.T
    elif kind == GEMM1:
        r = O - A @ B.T
    elif kind == POTRF:
        L = np.linalg.cholesky(np.tril(O) + np.tril(O, -1).T)
        pool[aux] = np.linalg.inv(L)
        pool[aux] = np.tril(pool[aux])
        r = L
    elif kind == TRSM1:
        r = O @ np.tril(B).T
    elif kind == TRTRI:
        r = B.copy()
    elif kind == TRMM2L:
        r = np.tril(A) @ O
    elif kind == GEMM2:
        r = O + A @ B
    elif kind == TRSM2R:
        r = -(O @ np.tril(B))
    elif kind == TRMM3:
        r = np.tril(A).T @ O
    elif kind == LAUUM:
        r = np.tril(O).T @ np.tril(O)
    elif kind == GEMM3:
        r = O + A.T @ B
    elif kind == SYRK3:
        r = O + A.T @ A
    else:
        raise ValueError(kind)
    pool[out] = r
    if cp >= 0:
        pool[cp] = r


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


def execute(plan, a, nb, order=None):
    t = plan["t"]
    pool = to_pool(a, t, nb)
    tasks = plan["tasks"]
    for v in (range(len(tasks)) if order is None else order):
        run_task(pool, tasks[v])
    return from_pool(pool, t, nb, a.shape[0])
