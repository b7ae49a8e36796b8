"""The FP64 inverse at the precision workload's orders, through the C-ABI.

At n >= 12288 (96 tiles per side and more) the library runs its default
large-order launch: two workgroups per CU and the step-1 chain products split
into row halves.  These tests run that launch at n = 16384 for the three
condition numbers of the precision workload, and once at n = 32768 (256
tiles per side, 1.35 million device tasks), against the analytic inverse
Q diag(1/lambda) Q^T of the construction A = Q diag(lambda) Q^T (a library
GEMM; the oracle would take hours at these orders).  The bar is the FP64
one, ||X - X_ref||_F / ||X_ref||_F <= 1e-12 kappa.  The launch shapes that
execute the same products in the same per-tile order (one workgroup per CU,
whole products, quarters instead of halves) must give the same bits."""
import pytest

import paper_1002_4057_amd as spd
from paper_1002_4057_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _err(x, ref):
    return (torch.linalg.norm(x - ref) / torch.linalg.norm(ref)).item()


def _resid(a, x):
    n = a.shape[0]
    eye = torch.eye(n, dtype=torch.float64, device=a.device)
    return (torch.linalg.norm(eye - a @ x) / torch.linalg.norm(a)).item()


@pytest.fixture(scope="module")
def q16384():
    q = inputs.orthogonal(16384, 0, device=DEV)
    yield q
    del q
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e10])
def test_default_launch_n16384_against_analytic_inverse(q16384, kappa):
    n = 16384
    a, lam = inputs.spectrum_from_q(q16384, kappa)
    x, rep = spd.spd_inverse(a, return_report=True)
    assert rep["info"] == 0 and rep["status"] == 0
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert rep["tiles"] == 128 and rep["workers"] == 2 * cus   # the large-order launch
    ref = inputs.analytic_inverse(q16384, lam)
    err = _err(x, ref)
    res = _resid(a, x)
    print(f"n={n} kappa={kappa:g}: rel err {err:.3e}, ||I-AX||_F/||A||_F {res:.3e}", flush=True)
    assert err <= 1e-12 * kappa
    # the stop rule of the precision workload is met by the FP64 form itself
    assert res <= 1e-13


def test_launch_shapes_bit_identical_n16384(q16384):
    """Default (512 workers, row halves, chains of 8) against one workgroup
    per CU, whole products, row quarters, and the chain lengths the
    autotuner chooses among (12 is its choice at this order): the same
    bits."""
    a, _ = inputs.spectrum_from_q(q16384, 1e6)
    x = spd.spd_inverse(a)
    for opts in (dict(per_cu=1), dict(no_split=1), dict(parts=4), dict(chain=12),
                 dict(chain=6, parts=2, per_cu=2)):
        assert torch.equal(x, spd.spd_inverse(a, **opts)), opts


def test_n32768_against_analytic_inverse():
    """The largest order of the precision workload: 256 x 256 tiles (13 GB of
    tile workspace), FP64, kappa = 1e2, in the launch the benchmark times."""
    n = 32768
    q = inputs.orthogonal(n, 0, device=DEV)
    a, lam = inputs.spectrum_from_q(q, 1e2)
    x, rep = spd.spd_inverse(a, return_report=True)
    assert rep["info"] == 0 and rep["status"] == 0 and rep["tiles"] == 256
    ref = inputs.analytic_inverse(q, lam)
    del q
    err = _err(x, ref)
    del ref
    res = _resid(a, x)
    print(f"n={n}: rel err {err:.3e}, ||I-AX||_F/||A||_F {res:.3e}, tasks {rep['tasks']}",
          flush=True)
    assert err <= 1e-12 * 1e2
    assert res <= 1e-13
    del a, x
    torch.cuda.empty_cache()
