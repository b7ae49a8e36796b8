"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only *generates* matrices; it holds none of the inversion
arithmetic and imports neither the GPU library nor the oracle.  Every
generator is deterministic for a given seed: random draws come from a CPU
``torch.Generator`` (float64), so the same seed gives the same numbers on any
machine.

Workload recipes (the paper has no datasets; all inputs are synthetic):

* ``wishart_shift``: B with iid N(0,1) entries, A = B B^T / n + s I
  (s = 1 for the single-matrix small case, s = 0.1 for the batched form).
* ``spectrum``: A = Q diag(lambda) Q^T with Q the orthogonal factor of a QR of
  an iid N(0,1) matrix and lambda_i = kappa^(i/(n-1)) (log-spaced over
  [1, kappa], endpoints included), symmetrised.  kappa_2(A) = kappa by
  construction, and Q diag(1/lambda) Q^T is the analytic inverse.
* ``tridiag``: tridiag(-1, 2, -1), whose Cholesky factor, factor inverse and
  inverse have closed forms.
* ``hilbert_scaled``: lcm(1..2n-1) * H (H the Hilbert matrix), an integer
  matrix whose inverse is H^{-1} / lcm, known exactly in rationals.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def randn(shape, seed: int) -> torch.Tensor:
    """iid N(0,1) float64 on the CPU from a seeded generator."""
    return torch.randn(*shape, generator=_gen(seed), dtype=torch.float64)


def wishart_shift(n: int, seed: int = 0, shift: float = 1.0) -> torch.Tensor:
    """A = B B^T / n + shift * I with B iid N(0,1) (CPU float64, symmetric)."""
    b = randn((n, n), seed)
    a = (b @ b.T) / n
    a = 0.5 * (a + a.T)
    a += shift * torch.eye(n, dtype=torch.float64)
    return a


def log_spectrum(n: int, kappa: float) -> torch.Tensor:
    """lambda_i = kappa^(i/(n-1)), i = 0..n-1 (float64)."""
    if n == 1:
        return torch.ones(1, dtype=torch.float64)
    e = torch.arange(n, dtype=torch.float64) / (n - 1)
    return torch.pow(torch.tensor(float(kappa), dtype=torch.float64), e)


def orthogonal(n: int, seed: int, device: str = "cpu") -> torch.Tensor:
    """Orthogonal Q from the QR of an iid N(0,1) matrix (seeded on the CPU)."""
    z = randn((n, n), seed).to(device)
    q, r = torch.linalg.qr(z)
    # fix the signs so that Q is a deterministic function of Z
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return q * s.unsqueeze(0)


def spectrum_from_q(q: torch.Tensor, kappa: float):
    """(A, lambda): A = Q diag(lambda) Q^T, lambda log-spaced over [1, kappa],
    for a given orthogonal Q (so that several condition numbers share one QR)."""
    lam = log_spectrum(q.shape[0], kappa).to(q.device)
    a = (q * lam.unsqueeze(0)) @ q.T
    a = 0.5 * (a + a.T)
    return a, lam


def spectrum(n: int, kappa: float, seed: int = 0, device: str = "cpu",
             return_factors: bool = False):
    """A = Q diag(lambda) Q^T with log-spaced lambda over [1, kappa]."""
    q = orthogonal(n, seed, device)
    a, lam = spectrum_from_q(q, kappa)
    if return_factors:
        return a, q, lam
    return a


def analytic_inverse(q: torch.Tensor, lam: torch.Tensor) -> torch.Tensor:
    """Q diag(1/lambda) Q^T for a ``spectrum`` matrix (library GEMM)."""
    x = (q * (1.0 / lam).unsqueeze(0)) @ q.T
    return 0.5 * (x + x.T)


def tridiag(n: int) -> np.ndarray:
    """tridiag(-1, 2, -1) of order n (float64)."""
    a = np.zeros((n, n), dtype=np.float64)
    idx = np.arange(n)
    a[idx, idx] = 2.0
    a[idx[1:], idx[:-1]] = -1.0
    a[idx[:-1], idx[1:]] = -1.0
    return a


def lcm_upto(m: int) -> int:
    v = 1
    for k in range(2, m + 1):
        v = v * k // math.gcd(v, k)
    return v


def hilbert_scaled(n: int):
    """(lcm * H as float64, lcm) with H_ij = 1/(i+j-1), 1-based."""
    s = lcm_upto(2 * n - 1)
    a = np.empty((n, n), dtype=np.float64)
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            a[i - 1, j - 1] = float(s // (i + j - 1))
    return a, s


def small_integer_spd(n: int, seed: int) -> np.ndarray:
    """A = M M^T + I with M entries uniform in {-2..2} (integer-valued float64)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(-2, 3, size=(n, n)).astype(np.int64)
    a = m @ m.T + np.eye(n, dtype=np.int64)
    return a.astype(np.float64)


def batch_orders(batch: int, lo: int, hi: int, seed: int) -> list:
    """Matrix orders drawn uniformly from {lo, ..., hi} (inclusive)."""
    g = _gen(seed)
    v = torch.randint(lo, hi + 1, (batch,), generator=g)
    return [int(x) for x in v.tolist()]


def batched_wishart(orders, seed: int, shift: float = 0.1):
    """A_i = B_i B_i^T / n_i + shift * I, one seed stream per matrix."""
    return [wishart_shift(n, seed=seed * 1000003 + i, shift=shift) for i, n in enumerate(orders)]
