"""GPU checks of the mixed-precision form (spd_inverse with mode
"mixed_fp32" through the C-ABI): FP32 tile DAG for X0, Newton-Schulz
refinement with binary64 residuals.

What pins it: the result against the FP64 oracle (or the analytic inverse)
at the FP64 bar 1e-12 * kappa; the stop rule ||I - A X||_F / ||A||_F <= tol
measured independently on the host; X0 really coming from FP32 arithmetic
(its residual is far above binary64 rounding); the quadratic convergence of
Newton-Schulz (each residual at most about the square of the previous plus
the binary64 floor); the fallback to FP64 when FP32 cannot start."""
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


def resid_rel(a, x):
    return np.linalg.norm(np.eye(a.shape[0]) - a @ x) / np.linalg.norm(a)


@pytest.mark.parametrize("n", [100, 129, 300, 513, 1000])
def test_mixed_against_oracle_kappa_1e2(n):
    a = inputs.spectrum(n, 1e2, seed=n).numpy()
    x, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32", return_report=True)
    x = x.cpu().numpy()
    ref = oracle.spd_inverse(a)
    err = rel_fro(x, ref)
    print(f"n={n}: rel err vs oracle {err:.3e}, iters {rep['refine_iters']}, "
          f"resid0 {rep['resid0_fro_rel']:.3e}, resid {rep['resid_fro_rel']:.3e}")
    assert rep["fell_back"] == 0
    assert err <= 1e-12 * 1e2
    assert resid_rel(a, x) <= 1e-13 * 4   # stop rule, re-measured on the host
    assert rep["resid_fro_rel"] <= 1e-13
    # X0 came from FP32 arithmetic: far above the binary64 residual, below 1
    assert 1e-10 < rep["resid0_fro_rel"] < 1e-2
    assert rep["refine_iters"] >= 1
    assert np.array_equal(x, x.T)


def test_refinement_is_quadratic():
    """R_{k+1} = I - A X_k (I + R_k) = R_k^2 exactly, so ||R_{k+1}||_F <=
    ||R_k||_F^2 up to rounding, until the binary64 floor (measured here at
    about 8e-15 relative; 5e-14 allowed)."""
    n = 640
    a = inputs.spectrum(n, 1e3, seed=3).numpy()
    res = []
    for k in range(0, 3):
        _, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32",
                                 return_report=True, max_refine=k + 1, refine_tol=1e-300,
                                 correction64=1)
        if k == 0:
            res.append(rep["resid0_fro_rel"])
        res.append(rep["resid_fro_rel"])
    anorm = np.linalg.norm(a)
    floor = 5e-14
    assert res[0] > 1e-9          # the FP32 start
    for r_prev, r_next in zip(res, res[1:]):
        assert r_next * anorm <= 4 * (r_prev * anorm) ** 2 + floor * anorm, res
    assert res[-1] <= floor, res


@pytest.mark.parametrize("n", [300, 1000, 2100])
def test_low_precision_corrections_against_oracle(n):
    """The default loop runs the corrections that another residual follows
    on the FP32 matrix cores and the last one in binary64: the result meets
    the stop rule and the FP64 bar against the oracle, as with every
    correction in binary64, in at most one more step."""
    a = inputs.spectrum(n, 1e2, seed=20 + n).numpy()
    ad = torch.from_numpy(a).to(DEV)
    x, rep = spd.spd_inverse(ad, mode="mixed_fp32", return_report=True)
    x64, rep64 = spd.spd_inverse(ad, mode="mixed_fp32", return_report=True, correction64=1)
    print(f"n={n}: {rep}\n  binary64 corrections: {rep64}", flush=True)
    assert rep["fell_back"] == 0 and rep["converged"] == 1
    assert rep["low_corrections"] >= 1 and rep64["low_corrections"] == 0
    assert rep["refine_iters"] <= rep64["refine_iters"] + 1
    x = x.cpu().numpy()
    assert rel_fro(x, oracle.spd_inverse(a)) <= 1e-12 * 1e2
    assert resid_rel(a, x) <= 1e-13
    assert np.array_equal(x, x.T)


def test_low_precision_step_within_its_rounding_bound():
    """One FP32 correction X1 = X0 + fl(X0 R0): I - A X1 = R0^2 - A E with E
    the rounding of the FP32 product (operands rounded to FP32, FP32
    accumulation over n terms), |E| <= (n + 4) u_32 |X0| |R0| entrywise, so
    ||I - A X1||_F <= ||R0||_F^2 + ||A||_2 (n + 4) u_32 ||X0||_F ||R0||_F
    (u_32 = 2^-24), up to the binary64 floor.  A product that dropped or
    transposed a term would leave a residual of the size of ||R0||_F."""
    n = 1000
    a = inputs.spectrum(n, 1e2, seed=21).numpy()
    ad = torch.from_numpy(a).to(DEV)
    x1, rep = spd.spd_inverse(ad, mode="mixed_fp32", return_report=True, max_refine=1,
                              refine_tol=1e-300)
    assert rep["low_corrections"] == 1 and rep["refine_iters"] == 1
    anorm = np.linalg.norm(a)
    r0 = rep["resid0_fro_rel"] * anorm
    x1 = x1.cpu().numpy()
    r1 = np.linalg.norm(np.eye(n) - a @ x1)
    xf = np.linalg.norm(x1)               # ||X0||_F to within ||X0 R0||_F
    bound = r0 ** 2 + 1e2 * (n + 4) * 2.0 ** -24 * xf * r0 + 64 * 2.0 ** -53 * anorm * xf
    print(f"r0 {r0:.3e}, r1 {r1:.3e}, bound {bound:.3e}")
    assert r1 <= bound
    assert r1 < 0.1 * r0


@pytest.mark.parametrize("n", [300, 1000, 2100])
def test_probe_estimate_tracks_the_measured_start_residual(n):
    """Before forming R0 = I - A X0 the library estimates ||R0||_F from 128
    random sign probes (E ||R0 V||_F^2 = 128 ||R0||_F^2, relative spread at
    most sqrt(2/128)): within a factor 1.5 of the measured value."""
    a = inputs.spectrum(n, 1e2, seed=40 + n).numpy()
    _, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32", return_report=True)
    print(rep, flush=True)
    assert rep["fell_back"] == 0
    ratio = rep["resid0_probe_rel"] / rep["resid0_fro_rel"]
    assert 1 / 1.5 <= ratio <= 1.5


def test_probe_rejects_a_hopeless_start_without_the_residual():
    """kappa = 1e7 at n = 2000: the FP32 start has ||R0||_F far above 1 (it
    grows with kappa: about 0.8 at kappa = 1e6 here); the probe estimate
    rejects it (reported in resid0_fro_rel, no residual formed) and the FP64
    path gives the result, bit for bit."""
    n = 2000
    a = torch.from_numpy(inputs.spectrum(n, 1e7, seed=41).numpy()).to(DEV)
    x, rep = spd.spd_inverse(a, mode="mixed_fp32", return_report=True)
    print(rep, flush=True)
    assert rep["fell_back"] == 1 and rep["refine_iters"] == 0
    anorm = torch.linalg.norm(a).item()
    assert rep["resid0_probe_rel"] * anorm > 2.0
    assert rep["resid0_fro_rel"] == rep["resid0_probe_rel"]
    assert rep["resid_last_rel"] == -1.0              # no residual was formed
    assert torch.equal(x, spd.spd_inverse(a))


def test_predicted_stop_skips_the_last_residual():
    """With the default tolerance the loop stops on the prediction
    ||I - A X'||_F <= ||R||_F^2 + floor (I - A (X + X R) = R^2), without
    forming the residual of the returned X; that residual, measured on the
    host, meets the stop rule."""
    n = 700
    a = inputs.spectrum(n, 1e2, seed=11).numpy()
    x, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32", return_report=True)
    print(rep)
    assert rep["fell_back"] == 0 and rep["converged"] == 1
    assert rep["predicted"] == 1 and rep["resid_fro_rel"] <= 1e-13
    assert rep["resid_last_rel"] > 1e-13          # the last residual formed was not enough
    assert resid_rel(a, x.cpu().numpy()) <= 1e-13  # the prediction held


def test_explicit_step_limit_returns_unconverged_result():
    """max_refine = 1 at the default tolerance: one step does not reach the
    stop rule; an explicit limit keeps the refined X and says so."""
    n = 500
    a = inputs.spectrum(n, 1e2, seed=12).numpy()
    x, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32", return_report=True,
                             max_refine=1)
    assert rep["fell_back"] == 0 and rep["converged"] == 0 and rep["refine_iters"] == 1
    assert rep["resid_fro_rel"] > 1e-13
    r = resid_rel(a, x.cpu().numpy())
    assert r > 1e-13 and r <= 4 * rep["resid_fro_rel"]   # the report does not claim convergence


def test_default_step_limit_exhausted_falls_back(monkeypatch):
    """When the library's own step limit runs out before the stop rule is met
    (forced from the host with a limit of one step), the FP64 path gives the
    result, bit for bit, with fell_back = 2."""
    n = 500
    a = torch.from_numpy(inputs.spectrum(n, 1e2, seed=12).numpy()).to(DEV)
    monkeypatch.setenv("SPDINV_DEFAULT_MAX_REFINE", "1")
    x, rep = spd.spd_inverse(a, mode="mixed_fp32", return_report=True)
    monkeypatch.delenv("SPDINV_DEFAULT_MAX_REFINE")
    assert rep["fell_back"] == 2 and rep["converged"] == 0
    assert torch.equal(x, spd.spd_inverse(a))


def test_tolerance_controls_iterations():
    n = 400
    a = torch.from_numpy(inputs.spectrum(n, 1e2, seed=5).numpy()).to(DEV)
    _, loose = spd.spd_inverse(a, mode="mixed_fp32", return_report=True, refine_tol=1e-2)
    _, tight = spd.spd_inverse(a, mode="mixed_fp32", return_report=True, refine_tol=1e-14)
    assert loose["refine_iters"] == 0 and loose["resid_fro_rel"] <= 1e-2
    assert tight["refine_iters"] > loose["refine_iters"]


def test_kappa_1e10_falls_back_to_fp64():
    n = 300
    a = inputs.spectrum(n, 1e10, seed=7).numpy()
    x, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32", return_report=True)
    assert rep["fell_back"] == 1
    ref = oracle.spd_inverse(a)
    assert rel_fro(x.cpu().numpy(), ref) <= 1e-12 * 1e10
    x64 = spd.spd_inverse(torch.from_numpy(a).to(DEV))
    assert torch.equal(x, x64)          # the FP64 path, bit for bit


def test_not_positive_definite_reports_info():
    n = 200
    a = inputs.wishart_shift(n, seed=8).numpy()
    a[150, 150] = -1.0
    with pytest.raises(spd.NotPositiveDefinite) as e:
        spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32")
    assert e.value.info == 151


@pytest.mark.parametrize("kappa", [1e2, 1e6])
def test_precision_workload_n16384(kappa):
    """The precision workload at n = 16384: A = Q diag(lambda) Q^T with lambda
    log-spaced over [1, kappa]; the result against the analytic inverse at the
    FP64 bar, and the stop rule on the device residual."""
    n = 16384
    a, q, lam = inputs.spectrum(n, kappa, seed=0, device=DEV, return_factors=True)
    x, rep = spd.spd_inverse(a, mode="mixed_fp32", return_report=True)
    ref = inputs.analytic_inverse(q, lam)
    err = (torch.linalg.norm(x - ref) / torch.linalg.norm(ref)).item()
    print(f"kappa={kappa:g}: err {err:.3e}, report {rep}")
    assert err <= 1e-12 * kappa
    if not rep["fell_back"]:
        assert rep["resid_fro_rel"] <= 1e-13


@pytest.mark.parametrize("n", [64, 300, 700])
def test_mixed_bf16_well_conditioned_against_oracle(n):
    """bfloat16 operands in the tile products: X0 carries a residual of the
    bfloat16 unit roundoff's order, far above the FP32 start, and the
    binary64 refinement still reaches the stop rule."""
    a = inputs.wishart_shift(n, seed=40 + n, shift=1.0).numpy()
    x, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_bf16", return_report=True)
    _, rep32 = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_fp32", return_report=True)
    ref = oracle.spd_inverse(a)
    ev = np.linalg.eigvalsh(a)
    err = rel_fro(x.cpu().numpy(), ref)
    print(f"bf16 n={n}: err {err:.3e}, report {rep}")
    assert rep["fell_back"] == 0
    assert rep["resid0_fro_rel"] > 30 * rep32["resid0_fro_rel"]   # bfloat16, not FP32, products
    assert rep["resid_fro_rel"] <= 1e-13
    assert err <= 1e-12 * ev[-1] / ev[0]


def test_mixed_bf16_kappa_1e2_result_within_fp64_bar():
    n = 513
    a = inputs.spectrum(n, 1e2, seed=41).numpy()
    x, rep = spd.spd_inverse(torch.from_numpy(a).to(DEV), mode="mixed_bf16", return_report=True)
    print(f"bf16 kappa=1e2: report {rep}")
    ref = oracle.spd_inverse(a)
    assert rel_fro(x.cpu().numpy(), ref) <= 1e-12 * 1e2
    if rep["fell_back"]:
        assert torch.equal(x, spd.spd_inverse(torch.from_numpy(a).to(DEV)))
    else:
        assert rep["resid_fro_rel"] <= 1e-13
