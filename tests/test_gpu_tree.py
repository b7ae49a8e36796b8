"""Tree reduction of the step-2 update chains on the GPU (spd_inverse and
spd_inverse_from_factor with opts.tree_levels, through the C-ABI).

Tolerance: relative Frobenius error <= 1e-12 * kappa(A) against the FP64
oracle, the bar of the FP64 path.  The tree is a fixed function of the tile
count (not of the schedule), so every worker count, chain length and grid
gives the same bits; partial renaming reads the same values from other
tiles, so it gives the bits of full renaming with the same tree."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def rel_fro(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def kappa(a):
    ev = np.linalg.eigvalsh(a)
    return ev[-1] / ev[0]


@pytest.mark.parametrize("n", [300, 1000, 2100])
@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("loop_order", [0, 1])
def test_tree_against_oracle(n, levels, loop_order):
    print(f"tree n={n} levels={levels} loop_order={loop_order}", flush=True)
    a = inputs.wishart_shift(n, seed=70 + n).numpy()
    x = spd.spd_inverse(torch.from_numpy(a).to(DEV), tree_levels=levels,
                        loop_order=loop_order).cpu().numpy()
    ref = oracle.spd_inverse(a)
    assert rel_fro(x, ref) <= 1e-12 * kappa(a)
    assert np.array_equal(x, x.T)


@pytest.mark.parametrize("levels", [1, 2])
def test_same_bits_for_every_schedule(levels):
    n = 3000
    print(f"tree schedules n={n} levels={levels}", flush=True)
    a = inputs.wishart_shift(n, seed=71).to(DEV)
    ref = spd.spd_inverse(a, tree_levels=levels)
    for opts in (dict(workers=37), dict(chain=1), dict(chain=12), dict(per_cu=1),
                 dict(no_split=1), dict(pipelined=0)):
        assert torch.equal(spd.spd_inverse(a, tree_levels=levels, **opts), ref), opts
    T = (-(-n // 128)) * (-(-n // 128) + 1) // 2
    assert torch.equal(spd.spd_inverse(a, tree_levels=levels, rename_tiles=T // 2), ref)
    # within rounding of the sequential chains
    seq = spd.spd_inverse(a)
    assert not torch.equal(seq, ref)
    k = kappa(a.cpu().numpy())
    assert (torch.linalg.norm(seq - ref) / torch.linalg.norm(seq)).item() <= 2e-12 * k


def test_in_place_tree_against_oracle():
    n = 1500
    print(f"tree in place n={n}", flush=True)
    a = inputs.wishart_shift(n, seed=72).numpy()
    for lo in (0, 1):
        x = spd.spd_inverse(torch.from_numpy(a).to(DEV), tree_levels=2, renamed=0, trtri_first=1,
                            loop_order=lo).cpu().numpy()
        assert rel_fro(x, oracle.spd_inverse(a)) <= 1e-12 * kappa(a)


@pytest.mark.parametrize("n", [129, 900, 1700])
def test_inverse_from_factor_with_tree(n):
    print(f"tree from factor n={n}", flush=True)
    a = inputs.wishart_shift(n, seed=73).numpy()
    lo = oracle.potrf(a)
    x = spd.inverse_from_factor(torch.from_numpy(lo).to(DEV), tree_levels=2).cpu().numpy()
    assert rel_fro(x, oracle.spd_inverse(a)) <= 1e-12 * kappa(a)


def test_large_tree_against_the_analytic_inverse():
    """n = 8193 (t = 65, a one-row ragged tile), UUU order: against the
    analytic inverse Q diag(1/lambda) Q^T of A = Q diag(lambda) Q^T (the
    oracle does not finish in seconds at this order)."""
    n, k = 8193, 1e4
    print(f"tree large n={n}", flush=True)
    a, q, lam = inputs.spectrum(n, k, seed=74, device=DEV, return_factors=True)
    ref = inputs.analytic_inverse(q, lam)
    for levels in (1, 2):
        x = spd.spd_inverse(a, tree_levels=levels, loop_order=1)
        err = (torch.linalg.norm(x - ref) / torch.linalg.norm(ref)).item()
        print(f"  levels={levels}: rel err {err:.3e}", flush=True)
        assert err <= 1e-12 * k
