"""GPU parity of the FP32 form of spd_inverse (SPDINV_FP32, through the
C-ABI): FP32 storage, tile products on the FP32 matrix cores with FP32
accumulation, diagonal tiles in binary64 rounded to FP32.

The reference is the oracle's binary64 inverse of the same FP32 input
(widened exactly).  Bar: the first-order error of an inverse computed with
unit roundoff u = 2^-24 through a Cholesky factor, (n + 4) u kappa_2(A): a
term linear in n for the products and a few roundings for the stored
inverted diagonal tiles and the stored result."""
import numpy as np
import pytest

import oracle
import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
U32 = 2.0 ** -24


def _check(a32, **opts):
    n = a32.shape[0]
    x = spd.spd_inverse(a32.to(DEV), mode="fp32", **opts)
    assert x.dtype == torch.float32
    an = a32.double().numpy()
    ref = oracle.spd_inverse(an)
    ev = np.linalg.eigvalsh(an)
    err = np.linalg.norm(x.cpu().double().numpy() - ref) / np.linalg.norm(ref)
    print(f"fp32 n={n}: rel err {err:.3e}", flush=True)
    assert err <= (n + 4) * U32 * ev[-1] / ev[0]
    return x


@pytest.mark.parametrize("n", [1, 5, 100, 128, 129, 300, 700, 1024])
def test_fp32_against_oracle(n):
    _check(inputs.wishart_shift(n, seed=40 + n).to(torch.float32))


def test_fp32_spectrum_kappa_1e3():
    a = inputs.spectrum(1000, 1e3, seed=3).to(torch.float32)
    _check(a)


def test_fp32_exact_identity_and_powers_of_two():
    d = torch.diag(torch.tensor([4.0 ** k for k in range(-3, 5)] * 20, dtype=torch.float32))
    x = spd.spd_inverse(d.to(DEV), mode="fp32")
    assert torch.equal(x.cpu(), torch.diag(1.0 / torch.diagonal(d)))


def test_fp32_info_and_untouched_upper():
    n = 300
    a = inputs.wishart_shift(n, seed=9).to(torch.float32)
    a[200, 200] = -50.0
    buf = a.t().contiguous().to(DEV)
    with pytest.raises(spd.NotPositiveDefinite) as e:
        spd.spd_inverse_(buf.t(), mode="fp32", report=True)
    assert e.value.info == 201
    # upper triangle untouched without fill_upper
    a = inputs.wishart_shift(n, seed=10).to(torch.float32)
    cm = a.t().contiguous()
    iu = torch.triu_indices(n, n, 1)
    cm[iu[1], iu[0]] = float("nan")     # column-major upper = row-major lower of cm
    buf = cm.to(DEV)
    spd.spd_inverse_(buf.t(), mode="fp32")
    out = buf.cpu()
    assert torch.isnan(out[iu[1], iu[0]]).all()
    assert not torch.isnan(torch.tril(out.t())).any()


@pytest.mark.parametrize("n", [700, 3000])
def test_fp32_workers_per_cu_do_not_change_the_bits(n):
    """One or two workgroups per CU (and a capped grid) run the same tasks
    with the same per-tile order of products: the same FP32 bits."""
    a32 = inputs.wishart_shift(n, seed=33).float().to(DEV)
    ref = spd.spd_inverse(a32, mode="fp32")
    for opts in (dict(per_cu=2), dict(per_cu=1), dict(workers=37)):
        assert torch.equal(spd.spd_inverse(a32, mode="fp32", **opts), ref), opts


@pytest.mark.parametrize("n", [700, 3000])
def test_fp32_chained_tasks_give_the_bits_of_single_products(n):
    """Chained FP32 products keep the accumulator in registers where separate
    tasks store and reload it (exact in FP32): the same bits for every chain
    length, single matrix and batched."""
    a32 = inputs.wishart_shift(n, seed=34).float().to(DEV)
    ref = spd.spd_inverse(a32, mode="fp32", chain=1)
    for c in (0, 4, 12):
        assert torch.equal(spd.spd_inverse(a32, mode="fp32", chain=c), ref), c
    mats = [inputs.wishart_shift(m, seed=35 + m).float().to(DEV) for m in (700, 300, 1500)]
    one = spd.batched_spd_inverse(mats, chain=1, batch_group=-1)
    for c in (4, 8):
        got = spd.batched_spd_inverse(mats, chain=c, batch_group=-1)
        assert all(torch.equal(x, y) for x, y in zip(got, one)), c
    assert torch.equal(one[2], spd.spd_inverse(mats[2], mode="fp32"))
