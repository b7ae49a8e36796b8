"""GPU parity of the backward of the inverse (spd_inverse_backward through the
C-ABI, and the autograd Function) against the FP64 oracle's gradient.

grad_A = -X S X with X = A^{-1}, S = (G + G^T)/2, formed as (X S) X -- the
same association as the oracle -- so with the oracle's X as input the two
results differ by at most the rounding of two length-n inner products each:
|d| <= 2 * 2 gamma_n (|X| |S| |X|) elementwise, gamma_n = n u / (1 - n u).
End to end (the GPU's own X) the bar is the forward's, relative Frobenius
error <= 1e-12 * kappa(A).  At the full size of the differentiation workload
(n = 4096) the check is central finite differences of the GPU forward on 64
seeded entries, a property that holds at any size."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
U = 2.0 ** -53


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gamma(n):
    return n * U / (1 - n * U)


def rel_fro(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


@pytest.mark.parametrize("n", [1, 2, 5, 127, 128, 129, 300, 640])
def test_backward_kernel_against_oracle_within_rounding_bound(n):
    a = inputs.wishart_shift(n, seed=n).numpy()
    x = oracle.spd_inverse(a)
    g = inputs.randn((n, n), seed=n + 1).numpy()
    ref = oracle.inverse_grad(x, g)
    got = spd.spd_inverse_backward(dev(x), dev(g)).cpu().numpy()
    s = 0.5 * (g + g.T)
    bound = 4.0 * gamma(n) * (np.abs(x) @ np.abs(s) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))
    assert np.array_equal(got, got.T)


def test_backward_identity_upstream_is_minus_inverse_squared():
    n = 257
    a = inputs.wishart_shift(n, seed=3).numpy()
    x = oracle.spd_inverse(a)
    got = spd.spd_inverse_backward(dev(x), dev(np.eye(n))).cpu().numpy()
    ref = -(x @ x)
    bound = 4.0 * gamma(n) * (np.abs(x) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(got - ref) <= bound)


def test_backward_depends_only_on_symmetric_part_bitwise():
    n = 200
    a = inputs.wishart_shift(n, seed=4).numpy()
    x = dev(oracle.spd_inverse(a))
    g = inputs.randn((n, n), seed=5).numpy()
    r1 = spd.spd_inverse_backward(x, dev(g)).cpu().numpy()
    r2 = spd.spd_inverse_backward(x, dev(g.T)).cpu().numpy()
    r3 = spd.spd_inverse_backward(x, dev(0.5 * (g + g.T))).cpu().numpy()
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)


def test_backward_uses_only_lower_triangle_of_x():
    n = 300
    a = inputs.wishart_shift(n, seed=6).numpy()
    x = oracle.spd_inverse(a)
    g = inputs.randn((n, n), seed=7).numpy()
    poisoned = np.tril(x) + np.triu(np.full((n, n), np.nan), 1)
    # the binding passes row-major storage as the column-major transpose:
    # the lower triangle of the column-major view is the upper of the tensor
    got = spd.spd_inverse_backward(dev(poisoned.T), dev(g)).cpu().numpy()
    ref = spd.spd_inverse_backward(dev(x), dev(g)).cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [200, 513])
def test_end_to_end_gradient_against_oracle(n):
    a = inputs.wishart_shift(n, seed=10 + n).numpy()
    g = inputs.randn((n, n), seed=11 + n).numpy()
    x_or = oracle.spd_inverse(a)
    ref = oracle.inverse_grad(x_or, g)
    at = dev(a).requires_grad_(True)
    x = spd.spd_inverse_ad(at)
    (x * dev(g)).sum().backward()
    got = at.grad.cpu().numpy()
    ev = np.linalg.eigvalsh(a)
    assert rel_fro(got, ref) <= 1e-12 * ev[-1] / ev[0]
    assert rel_fro(x.detach().cpu().numpy(), x_or) <= 1e-12 * ev[-1] / ev[0]


def test_gradcheck_small():
    n = 6
    a0 = inputs.wishart_shift(n, seed=20).to(DEV)
    a = a0.clone().requires_grad_(True)

    def f(m):
        return spd.spd_inverse_ad(0.5 * (m + m.t()))

    assert torch.autograd.gradcheck(f, (a,), eps=1e-6, atol=1e-7, rtol=1e-5)


def _fd_entries(n, count, seed):
    gen = torch.Generator().manual_seed(seed)
    p = torch.randint(0, n, (count,), generator=gen).tolist()
    q = torch.randint(0, n, (count,), generator=gen).tolist()
    return [(max(i, j), min(i, j)) for i, j in zip(p, q)]


def _loss(a_dev, g_dev):
    x = spd.spd_inverse(a_dev)
    return torch.sum(g_dev * x).item()


def test_finite_differences_full_size_n4096():
    """Differentiation workload (a): n = 4096, A = B B^T/n + I, G iid N(0,1)
    (seed 1), central differences with h = 1e-6 in symmetric directions on
    64 seeded entries (seed 2)."""
    n, h = 4096, 1e-6
    a = inputs.wishart_shift(n, seed=0).to(DEV)
    g = inputs.randn((n, n), seed=1).to(DEV)
    at = a.clone().requires_grad_(True)
    x = spd.spd_inverse_ad(at)
    (x * g).sum().backward()
    grad = at.grad
    errs = []
    for (p, q) in _fd_entries(n, 64, seed=2):
        ap, am = a.clone(), a.clone()
        # the forward reads the lower triangle: moving entry (p, q), p >= q,
        # moves both (p, q) and (q, p) of the symmetric matrix
        ap[p, q] += h
        am[p, q] -= h
        fd = (_loss(ap, g) - _loss(am, g)) / (2 * h)
        an = (2.0 if p != q else 1.0) * grad[p, q].item()
        errs.append(abs(fd - an))
        assert abs(fd - an) <= 1e-5 * abs(an) + 2e-6, (p, q, fd, an)
    assert max(errs) < 2e-6


def test_batched_small_matrices_against_oracle():
    """Differentiation workload (b): 256 matrices of n = 256 built as the
    small single-matrix case, forward + backward through the autograd
    Function, every gradient against the oracle's."""
    n, batch = 256, 256
    a = torch.stack([inputs.wishart_shift(n, seed=1000 + i) for i in range(batch)])
    g = torch.stack([inputs.randn((n, n), seed=5000 + i) for i in range(batch)])
    at = a.to(DEV).requires_grad_(True)
    x = spd.spd_inverse_ad(at)
    (x * g.to(DEV)).sum().backward()
    got = at.grad.cpu().numpy()
    an, gn = a.numpy(), g.numpy()
    worst = 0.0
    for i in range(batch):
        x_or = oracle.spd_inverse(an[i])
        ref = oracle.inverse_grad(x_or, gn[i])
        ev = np.linalg.eigvalsh(an[i])
        r = rel_fro(got[i], ref) / (1e-12 * ev[-1] / ev[0])
        worst = max(worst, r)
    assert worst <= 1.0, worst


# ---- batched backward (batched_spd_inverse_backward, one launch) ----------
def test_batched_backward_matches_single_calls_and_oracle():
    """Uneven orders in one launch: each gradient is the single-matrix
    kernel's bit for bit (same tile products in the same order) and within
    the rounding bound of the oracle's gradient."""
    orders = [1, 5, 100, 128, 129, 300, 700, 0, 256]
    xs, gs, refs = [], [], []
    for k, n in enumerate(orders):
        a = inputs.wishart_shift(n, seed=70 + k).numpy() if n else np.zeros((0, 0))
        x = oracle.spd_inverse(a) if n else a
        g = inputs.randn((n, n), seed=80 + k).numpy() if n else a
        xs.append(dev(x))
        gs.append(dev(g))
        refs.append(oracle.inverse_grad(x, g) if n else a)
    got = spd.batched_spd_inverse_backward(xs, gs)
    for n, x, g, r, y in zip(orders, xs, gs, refs, got):
        if n == 0:
            continue
        assert torch.equal(y, spd.spd_inverse_backward(x, g)), n
        xn, gn = x.cpu().numpy(), g.cpu().numpy()
        s = 0.5 * (gn + gn.T)
        bound = 4.0 * gamma(n) * (np.abs(xn) @ np.abs(s) @ np.abs(xn)) + 1e-300
        assert np.all(np.abs(y.cpu().numpy() - r) <= bound), n


def test_batched_backward_workload_256_of_256():
    """Differentiation workload (b): 256 matrices of n = 256 in one launch,
    every gradient against the single-matrix call, 8 against the oracle."""
    n, batch = 256, 256
    a = torch.stack([inputs.wishart_shift(n, seed=900 + k) for k in range(batch)]).to(DEV)
    x = torch.stack(spd.batched_spd_inverse(list(a)))
    g = torch.stack([inputs.randn((n, n), seed=2000 + k) for k in range(batch)]).to(DEV)
    got = spd.batched_spd_inverse_backward(list(x), list(g))
    for k in range(batch):
        assert torch.equal(got[k], spd.spd_inverse_backward(x[k], g[k])), k
    for k in range(0, batch, 32):
        xn, gn = x[k].cpu().numpy(), g[k].cpu().numpy()
        ref = oracle.inverse_grad(xn, gn)
        assert rel_fro(got[k].cpu().numpy(), ref) <= 1e-12


def test_autograd_batched_branch_uses_the_batched_launches():
    """SpdInverse on a (B, n, n) tensor: forward by batched_spd_inverse,
    backward by batched_spd_inverse_backward; the gradient equals the
    per-matrix autograd gradient."""
    n, batch = 150, 12
    a = torch.stack([inputs.wishart_shift(n, seed=300 + k) for k in range(batch)]).to(DEV)
    g = torch.stack([inputs.randn((n, n), seed=400 + k) for k in range(batch)]).to(DEV)
    ab = a.clone().requires_grad_(True)
    (spd.spd_inverse_ad(ab) * g).sum().backward()
    for k in range(batch):
        ak = a[k].clone().requires_grad_(True)
        (spd.spd_inverse_ad(ak) * g[k]).sum().backward()
        assert torch.equal(ab.grad[k], ak.grad), k
