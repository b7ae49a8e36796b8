"""The allocation-free entry point (spd_inverse_noalloc) through the C-ABI.

It runs the plan and kernels of spd_inverse with the workspace and the plan's
device tables in the library's per-GPU scratch array, so its result must be
bit-identical to spd_inverse's with a caller workspace.  Two calls in a row,
the second on a smaller matrix (the scratch keeps the first call's contents),
then orders past the stated maximum, which must be rejected on the host."""
import ctypes

import pytest

import paper_1002_4057_amd as spd
from paper_1002_4057_amd import _lib, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _colmajor(a):
    return a.t().contiguous()          # storage of a read column-major (a symmetric)


def _reference(a_cm, **opts):
    ref = a_cm.clone()
    spd.spd_inverse_(ref.t(), **opts)
    return ref


def _noalloc(a_cm, **opts):
    out = a_cm.clone()
    info = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    lib = _lib.load()
    o = _lib.make_opts(**opts)
    n = a_cm.shape[0]
    rc = lib.spd_inverse_noalloc(n, out.data_ptr(), n,
                                 torch.cuda.current_stream().cuda_stream, ctypes.byref(o),
                                 info.data_ptr())
    assert rc == 0
    torch.cuda.synchronize()
    return out, int(info.item())


def test_two_calls_match_spd_inverse_bit_for_bit():
    a1 = _colmajor(inputs.wishart_shift(1500, seed=11).to(DEV))   # 12 tiles, ragged
    a2 = _colmajor(inputs.wishart_shift(700, seed=12).to(DEV))    # 6 tiles, ragged
    print("noalloc: n=1500 then n=700", flush=True)
    r1 = _reference(a1)
    x1, info1 = _noalloc(a1)
    assert info1 == 0
    assert torch.equal(x1, r1)
    r2 = _reference(a2)
    x2, info2 = _noalloc(a2)
    assert info2 == 0
    assert torch.equal(x2, r2)
    # and back to the first plan (the scratch's tables are replaced again)
    x3, _ = _noalloc(a1)
    assert torch.equal(x3, r1)


def test_largest_order_and_options_match():
    n = _lib.NOALLOC_MAX_N
    a = _colmajor(inputs.wishart_shift(n, seed=13).to(DEV))
    print(f"noalloc: n={n}", flush=True)
    r = _reference(a, fill_upper=1)
    x, info = _noalloc(a, fill_upper=1)
    assert info == 0 and torch.equal(x, r)
    small = _colmajor(inputs.wishart_shift(300, seed=14).to(DEV))
    r = _reference(small, chain=1)
    x, info = _noalloc(small, chain=1)
    assert info == 0 and torch.equal(x, r)


def test_not_positive_definite_reports_info():
    n = 260
    a = torch.eye(n, dtype=torch.float64, device=DEV)
    a[200, 200] = -1.0
    _, info = _noalloc(a.contiguous())
    assert info == 201


def test_orders_past_the_maximum_are_rejected():
    lib = _lib.load()
    n = _lib.NOALLOC_MAX_N + 1
    buf = torch.zeros(4, dtype=torch.float64, device=DEV)
    before = buf.clone()
    rc = lib.spd_inverse_noalloc(n, buf.data_ptr(), n, None, None, None)
    assert rc == -1
    torch.cuda.synchronize()
    assert torch.equal(buf, before)
