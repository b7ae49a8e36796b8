"""Mutation check of the oracle's pins (CPU only).

Plausible mistakes (a dropped term, a wrong sign, a wrong index, a transposed
operand, reading the wrong triangle) are planted in temporary copies of the
oracle's C source.  Each mutant is compiled and run against the pins of
``test_oracle``; every mutant must fail at least one pin.  This shows that the
pins constrain each stage of the oracle, rather than the oracle agreeing with
itself.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1002_4057_amd import inputs
from test_oracle import (U, gauss_jordan_inverse, hilbert_inverse_exact, rel_fro,
                         tridiag_inv, tridiag_L, tridiag_Linv)

SRC = os.path.join(os.path.dirname(oracle.__file__), "spd_oracle.c")

# (name, original text, replacement) -- each original must occur exactly once
MUTANTS = [
    ("chol_drop_diag_term", "for (int k = 0; k < j; ++k) d -= lj[k] * lj[k];",
     "for (int k = 0; k + 1 < j; ++k) d -= lj[k] * lj[k];"),
    ("chol_sign", "s -= li[k] * lj[k];", "s += li[k] * lj[k];"),
    ("chol_wrong_index", "s -= li[k] * lj[k];", "s -= li[k] * li[k];"),
    ("chol_scale_op", "Lr[(size_t)i * n + j] = s / ljj;", "Lr[(size_t)i * n + j] = s * ljj;"),
    ("chol_reads_upper", "double s = CM(A, lda, i, j);", "double s = CM(A, lda, j, i);"),
    ("trtri_drop_term", "for (int k = j + 1; k <= i; ++k) s += xi[k] * lcol[k];",
     "for (int k = j + 1; k < i; ++k) s += xi[k] * lcol[k];"),
    ("trtri_sign", "Xr[(size_t)i * n + j] = -s / ljj;", "Xr[(size_t)i * n + j] = s / ljj;"),
    ("trtri_transposed_operand", "s += xi[k] * lcol[k];", "s += xi[k] * Lc[(size_t)k * n + j];"),
    ("trtri_diag_divisor", "Xr[(size_t)i * n + j] = -s / ljj;",
     "Xr[(size_t)i * n + j] = -s / Lc[(size_t)i * n + i];"),
    ("lauum_drop_term", "for (int k = i; k < n; ++k) s += xi[k] * xj[k];",
     "for (int k = i + 1; k < n; ++k) s += xi[k] * xj[k];"),
    ("lauum_wrong_index", "s += xi[k] * xj[k];", "s += xi[k] * xi[k];"),
    ("lauum_drop_last_term", "for (int k = i; k < n; ++k) s += xi[k] * xj[k];",
     "for (int k = i; k + 1 < n; ++k) s += xi[k] * xj[k];"),
    ("grad_no_symmetrise", "(CM(G, ldg, i, j) + CM(G, ldg, j, i)) / 2.0", "CM(G, ldg, i, j)"),
    ("grad_sign", "CM(grad, ldgr, i, j) = -s;", "CM(grad, ldgr, i, j) = s;"),
    ("grad_transposed_Y", "const double y = (i >= j) ? CM(Ylow, ldy, i, j) : CM(Ylow, ldy, j, i);",
     "const double y = CM(Ylow, ldy, i, j);"),
]


def _battery(o):
    """Run the pins on an oracle build; return the names of those that fail."""
    failed = []

    def check(name, fn):
        try:
            if not fn():
                failed.append(name)
        except Exception:
            failed.append(name)

    for n in (7, 16):
        check(f"tridiag_L_{n}", lambda: np.abs(o.potrf(inputs.tridiag(n)) - tridiag_L(n)).max() <= 8 * n * U)
        check(f"tridiag_X_{n}", lambda: rel_fro(o.trtri(tridiag_L(n)), tridiag_Linv(n)) <= 16 * n * U)
        check(f"tridiag_Y_{n}", lambda: rel_fro(o.lauum(tridiag_Linv(n)), np.tril(tridiag_inv(n))) <= 16 * n * U)
        check(f"tridiag_inv_{n}", lambda: rel_fro(o.spd_inverse(inputs.tridiag(n)), tridiag_inv(n)) <= 1e-12)
    a, s = inputs.hilbert_scaled(5)
    check("hilbert_5", lambda: rel_fro(o.spd_inverse(a), np.array(hilbert_inverse_exact(5)) / s)
          <= 32 * 5 * U * np.linalg.cond(a))
    b = inputs.small_integer_spd(7, 3)
    check("gauss_jordan_7", lambda: rel_fro(o.spd_inverse(b), np.array(gauss_jordan_inverse(b)))
          <= 16 * 7 * U * np.linalg.cond(b))
    d = 4.0 ** np.array([-3, 0, 2, 5, -1])
    check("diag_exact", lambda: np.array_equal(o.spd_inverse(np.diag(d)), np.diag(1.0 / d)))
    w = inputs.wishart_shift(12, seed=11).numpy()
    p = w.copy()
    p[np.triu_indices(12, 1)] = np.nan
    check("upper_never_read", lambda: np.all(np.isfinite(np.tril(o.spd_inverse_lower(p)))))
    dg = np.array([1.5, 2.0, 0.25, 4.0])
    g = inputs.randn((4, 4), seed=1).numpy()
    check("grad_diag", lambda: np.allclose(o.inverse_grad(np.diag(1.0 / dg), g),
                                           -0.5 * (g + g.T) / np.outer(dg, dg), rtol=1e-14, atol=0))

    def grad_fd():
        n = 6
        aa = inputs.wishart_shift(n, seed=5).numpy()
        gg = inputs.randn((n, n), seed=1).numpy()
        grad = o.inverse_grad(o.spd_inverse(aa), gg)
        for (pp, qq) in [(3, 1), (5, 5), (4, 0)]:
            e = np.zeros((n, n))
            e[pp, qq] += 1.0
            if pp != qq:
                e[qq, pp] += 1.0
            h = 1e-6
            fd = (math.fsum((gg * o.spd_inverse(aa + h * e)).ravel())
                  - math.fsum((gg * o.spd_inverse(aa - h * e)).ravel())) / (2 * h)
            an = grad[pp, qq] * (2.0 if pp != qq else 1.0)
            if abs(fd - an) > 1e-6 * max(1.0, abs(an)):
                return False
        return True

    check("grad_fd", grad_fd)

    def grad_lower_only():
        n = 5
        yy = o.spd_inverse(inputs.wishart_shift(n, seed=6).numpy())
        gg = inputs.randn((n, n), seed=2).numpy()
        low = np.tril(yy)
        low[np.triu_indices(n, 1)] = np.nan
        return np.array_equal(o.inverse_grad(low, gg), o.inverse_grad(yy, gg))

    check("grad_lower_only", grad_lower_only)
    return failed


def test_unmutated_oracle_passes_battery():
    assert _battery(oracle) == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
                           str(mutated), "-o", str(so), "-lm"])
    failed = _battery(oracle.load_variant(str(so)))
    assert failed, f"mutant {name} passed every pin"
