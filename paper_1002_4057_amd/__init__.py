"""MI355X-native tile inversion of symmetric positive definite matrices.

The package is a thin Python layer over ``libspdinv.so`` (C-ABI in
``include/spdinv.h``).  PyTorch provides device memory and streams; every
step of the inversion runs in the library's HIP kernels.

Main entry points
-----------------
``spd_inverse(a)``      full symmetric A^{-1} of a CUDA float64 tensor
``spd_inverse_(a_cm)``  in place on a column-major view (lower triangle)
``batched_spd_inverse(mats)``   many uneven matrices in one persistent launch
``spd_inverse_backward(x, g)``  -X sym(G) X, the adjoint of the inverse
``SpdInverse.apply(a)`` autograd Function (forward + backward on the GPU)
``plan_stats(t)``       planner statistics (critical paths of Table 1)
``plan_export(t)``      the task DAG the device executes
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import LibraryNotBuilt, load, make_opts, TASK_NAMES  # noqa: F401

__all__ = ["spd_inverse", "spd_inverse_", "workspace_bytes", "plan_stats", "plan_export",
           "spd_inverse_backward", "backward_workspace_bytes", "SpdInverse", "spd_inverse_ad",
           "batched_spd_inverse", "batched_spd_inverse_", "batched_workspace_bytes",
           "cholesky", "cholesky_", "inverse_from_factor", "inverse_from_factor_",
           "solve", "solve_", "solve_from_factor", "solve_from_factor_", "solve_workspace_bytes",
           "spd_inverse_noalloc_", "batched_spd_inverse_backward",
           "batched_backward_workspace_bytes", "batched_spd_inverse_backward_", "autotune", "autotune_batched", "tuning_save",
           "tuning_load", "tuning_clear", "SpdInverseError", "NotPositiveDefinite"]


class SpdInverseError(RuntimeError):
    pass


class NotPositiveDefinite(SpdInverseError):
    def __init__(self, info: int):
        super().__init__(f"leading minor of order {info} is not positive definite")
        self.info = info


def _stream_ptr(device) -> int:
    import torch
    return torch.cuda.current_stream(device).cuda_stream


MODES = {"fp64": _lib.SPDINV_FP64, "fp32": _lib.SPDINV_FP32, "mixed_fp32": _lib.SPDINV_MIXED_FP32,
         "mixed_bf16": _lib.SPDINV_MIXED_BF16}


def _dtype_of(mode: str):
    import torch
    return torch.float32 if mode == "fp32" else torch.float64


def _mode(mode) -> int:
    try:
        return MODES[mode]
    except KeyError:
        raise ValueError(f"mode must be one of {sorted(MODES)}") from None


def workspace_bytes(n: int, mode: str = "fp64", **opts) -> int:
    o = make_opts(**opts)
    return int(load().spd_inverse_workspace_bytes(int(n), _mode(mode), ctypes.byref(o)))


def spd_inverse_(a_cm, *, mode: str = "fp64", work=None, report: bool = False, info=None,
                 **opts):
    """A <- A^{-1} in place on a column-major CUDA view (float64; float32 for
    mode "fp32").

    ``a_cm`` must have strides (1, ld) with ld >= n (e.g. ``x.t()`` of a
    row-major tensor).  Its lower triangle in column-major indexing, i.e.
    ``a_cm[i, j]`` for i >= j, is read and replaced.  ``work`` may be a
    preallocated uint8 CUDA tensor of at least ``workspace_bytes`` bytes.
    ``info`` may be a CUDA int32 tensor of one element receiving INFO.  With
    ``report=True`` the call synchronises and returns the library report as a
    dict (raising NotPositiveDefinite on INFO > 0).  ``mode`` is "fp64",
    "fp32" (FP32 storage and tile products, binary64 diagonal tiles, no
    refinement), "mixed_fp32" (FP32 tile DAG + binary64 Newton-Schulz
    refinement; the report then carries refine_iters, fell_back and the
    relative residuals) or "mixed_bf16" (the same with bfloat16 operands in
    the tile products).
    """
    import torch
    want = _dtype_of(mode)
    if a_cm.dtype != want or not a_cm.is_cuda or a_cm.dim() != 2:
        raise TypeError(f"expected a 2-D CUDA {want} tensor")
    n = a_cm.shape[0]
    if a_cm.shape[1] != n:
        raise ValueError("matrix must be square")
    if n > 1 and a_cm.stride(0) != 1:
        raise ValueError("expected a column-major view (stride(0) == 1)")
    lda = max(1, a_cm.stride(1) if n > 1 else max(1, n))
    lib = load()
    o = make_opts(**opts)
    m = _mode(mode)
    need = int(lib.spd_inverse_workspace_bytes(n, m, ctypes.byref(o)))
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=a_cm.device)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    rep = _lib.Report()
    info_ptr = info.data_ptr() if info is not None else None
    rc = lib.spd_inverse(n, a_cm.data_ptr(), lda, m, work.data_ptr(), need,
                         _stream_ptr(a_cm.device), ctypes.byref(o), info_ptr,
                         ctypes.byref(rep) if report else None)
    if rc != 0:
        raise SpdInverseError(f"spd_inverse returned {rc}")
    if report:
        r = {f: getattr(rep, f) for f, _ in _lib.Report._fields_}
        if r["info"] > 0:
            raise NotPositiveDefinite(r["info"])
        return r
    return None


def spd_inverse_noalloc_(a_cm, *, info=None, **opts):
    """A <- A^{-1} in place on a column-major CUDA float64 view, as
    ``spd_inverse_`` in FP64, through the library's allocation-free entry
    point: no workspace argument (the library's per-GPU device scratch holds
    it), n <= 2048, asynchronous on the current stream.  Calls that may
    overlap on one GPU race."""
    import torch
    if a_cm.dtype != torch.float64 or not a_cm.is_cuda or a_cm.dim() != 2:
        raise TypeError("expected a 2-D CUDA float64 tensor")
    n = a_cm.shape[0]
    if a_cm.shape[1] != n:
        raise ValueError("matrix must be square")
    if n > 1 and a_cm.stride(0) != 1:
        raise ValueError("expected a column-major view (stride(0) == 1)")
    lda = max(1, a_cm.stride(1) if n > 1 else max(1, n))
    o = make_opts(**opts)
    rc = load().spd_inverse_noalloc(n, a_cm.data_ptr(), lda, _stream_ptr(a_cm.device),
                                    ctypes.byref(o), info.data_ptr() if info is not None else None)
    if rc != 0:
        raise SpdInverseError(f"spd_inverse_noalloc returned {rc}")


def _fp64_step_entry(name: str, a_cm, work, report: bool, info, opts):
    import torch
    if a_cm.dtype != torch.float64 or not a_cm.is_cuda or a_cm.dim() != 2:
        raise TypeError("expected a 2-D CUDA float64 tensor")
    n = a_cm.shape[0]
    if a_cm.shape[1] != n:
        raise ValueError("matrix must be square")
    if n > 1 and a_cm.stride(0) != 1:
        raise ValueError("expected a column-major view (stride(0) == 1)")
    lda = max(1, a_cm.stride(1) if n > 1 else max(1, n))
    lib = load()
    o = make_opts(**opts)
    need = int(lib.spd_inverse_workspace_bytes(n, _lib.SPDINV_FP64, ctypes.byref(o)))
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=a_cm.device)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    rep = _lib.Report()
    info_ptr = info.data_ptr() if info is not None else None
    rc = getattr(lib, name)(n, a_cm.data_ptr(), lda, work.data_ptr(), need,
                            _stream_ptr(a_cm.device), ctypes.byref(o), info_ptr,
                            ctypes.byref(rep) if report else None)
    if rc != 0:
        raise SpdInverseError(f"{name} returned {rc}")
    if report:
        r = {f: getattr(rep, f) for f, _ in _lib.Report._fields_}
        if r["info"] > 0:
            raise NotPositiveDefinite(r["info"])
        return r
    return None


def cholesky_(a_cm, *, work=None, report: bool = False, info=None, **opts):
    """A <- L (A = L L^T) in place on the lower triangle of a column-major
    CUDA float64 view (step 1 of Algorithm 1 alone); the strictly upper
    triangle is left as it is.  Arguments as for spd_inverse_ (FP64 only)."""
    return _fp64_step_entry("spd_cholesky", a_cm, work, report, info, opts)


def cholesky(a, return_report: bool = False, **opts):
    """Lower Cholesky factor L of a CUDA float64 SPD tensor (lower triangle
    read), with zeros above the diagonal."""
    import torch
    n = a.shape[-1]
    buf = a.t().contiguous()
    rep = cholesky_(buf.t(), report=True, **opts) if n else None
    l = torch.tril(buf.t()).contiguous() if n else torch.empty_like(a)
    return (l, rep) if return_report else l


def inverse_from_factor_(l_cm, *, work=None, report: bool = False, info=None, **opts):
    """L <- (L L^T)^{-1} in place: the lower triangle of a column-major CUDA
    float64 view holds the Cholesky factor on entry and the lower triangle of
    the inverse on exit (steps 2 and 3 of Algorithm 1).  INFO = k > 0 when
    L_kk = 0.  Arguments as for spd_inverse_ (FP64 only)."""
    return _fp64_step_entry("spd_inverse_from_factor", l_cm, work, report, info, opts)


def inverse_from_factor(l, return_report: bool = False, **opts):
    """Full symmetric (L L^T)^{-1} from a CUDA float64 lower Cholesky factor L
    (its strictly upper triangle is not read)."""
    import torch
    n = l.shape[-1]
    buf = l.t().contiguous()
    rep = inverse_from_factor_(buf.t(), report=True, fill_upper=1, **opts) if n else None
    x = buf.t().contiguous() if n else torch.empty_like(l)
    return (x, rep) if return_report else x


def _colmajor_check(x, rows=None):
    import torch
    if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 2:
        raise TypeError("expected a 2-D CUDA float64 tensor")
    if rows is not None and x.shape[0] != rows:
        raise ValueError("row count does not match the matrix order")
    if x.shape[0] > 1 and x.shape[1] > 0 and x.stride(0) != 1:
        raise ValueError("expected a column-major view (stride(0) == 1)")
    return max(1, x.stride(1) if x.shape[0] > 1 and x.shape[1] > 1 else max(1, x.shape[0]))


def _solve_entry(name, a_cm, b_cm, work, report, info, opts):
    import torch
    n = a_cm.shape[0]
    if a_cm.shape[1] != n:
        raise ValueError("matrix must be square")
    lda = _colmajor_check(a_cm)
    ldb = _colmajor_check(b_cm, rows=n)
    nrhs = b_cm.shape[1]
    lib = load()
    o = make_opts(**opts)
    need = int(lib.spd_solve_workspace_bytes(n, nrhs, ctypes.byref(o)))
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=a_cm.device)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    rep = _lib.Report()
    info_ptr = info.data_ptr() if info is not None else None
    rc = getattr(lib, name)(n, nrhs, a_cm.data_ptr(), lda, b_cm.data_ptr(), ldb,
                            work.data_ptr(), need, _stream_ptr(a_cm.device), ctypes.byref(o),
                            info_ptr, ctypes.byref(rep) if report else None)
    if rc != 0:
        raise SpdInverseError(f"{name} returned {rc}")
    if report:
        r = {f: getattr(rep, f) for f, _ in _lib.Report._fields_}
        if r["info"] > 0:
            raise NotPositiveDefinite(r["info"])
        return r
    return None


def solve_workspace_bytes(n: int, nrhs: int, **opts) -> int:
    """Device workspace bytes of spd_solve / spd_solve_from_factor."""
    o = make_opts(**opts)
    return int(load().spd_solve_workspace_bytes(int(n), int(nrhs), ctypes.byref(o)))


def solve_(a_cm, b_cm, *, work=None, report: bool = False, info=None, **opts):
    """A X = B in place on column-major CUDA float64 views (as xPOSV): the
    lower triangle of A is replaced by its Cholesky factor L and B (n x nrhs)
    by X."""
    return _solve_entry("spd_solve", a_cm, b_cm, work, report, info, opts)


def solve(a, b, return_report: bool = False, **opts):
    """X with A X = B for a CUDA float64 SPD A (lower triangle read) and a
    CUDA float64 B of shape (n, nrhs); A and B are not modified."""
    abuf = a.t().contiguous()
    bbuf = b.t().contiguous()
    rep = solve_(abuf.t(), bbuf.t(), report=True, **opts) if a.shape[-1] else None
    x = bbuf.t().contiguous()
    return (x, rep) if return_report else x


def solve_from_factor_(l_cm, b_cm, *, work=None, report: bool = False, info=None, **opts):
    """L L^T X = B in place on column-major CUDA float64 views (as xPOTRS):
    the lower triangle of L holds the factor (only read); B is replaced by X."""
    return _solve_entry("spd_solve_from_factor", l_cm, b_cm, work, report, info, opts)


def solve_from_factor(l, b, return_report: bool = False, **opts):
    """X with L L^T X = B for a CUDA float64 lower Cholesky factor L."""
    lbuf = l.t().contiguous()
    bbuf = b.t().contiguous()
    rep = solve_from_factor_(lbuf.t(), bbuf.t(), report=True, **opts) if l.shape[-1] else None
    x = bbuf.t().contiguous()
    return (x, rep) if return_report else x


def spd_inverse(a, mode: str = "fp64", return_report: bool = False, **opts):
    """Full symmetric A^{-1} of a CUDA float64 tensor (float32 for mode
    "fp32"); the lower triangle is read."""
    import torch
    n = a.shape[-1]
    buf = a.t().contiguous()          # column-major storage of a: lower triangle = a's lower
    rep = spd_inverse_(buf.t(), mode=mode, fill_upper=1, report=True, **opts) if n else None
    x = buf.t().contiguous() if n else torch.empty_like(a)
    return (x, rep) if return_report else x


def _int_array(values):
    arr = (ctypes.c_int * max(1, len(values)))(*[int(v) for v in values])
    return arr


def batched_workspace_bytes(orders, mode: str = "fp64", **opts) -> int:
    o = make_opts(**opts)
    arr = _int_array(orders)
    return int(load().batched_spd_inverse_workspace_bytes(len(orders), arr, _batched_mode(mode),
                                                          ctypes.byref(o)))


def _batched_mode(mode: str) -> int:
    if mode not in ("fp64", "fp32"):
        raise ValueError("batched mode must be 'fp64' or 'fp32'")
    return MODES[mode]


def batched_spd_inverse_(ptrs, orders, n_dev, lda_dev, *, mode: str = "fp64", work=None,
                         info=None, **opts):
    """Low-level batched call: ``ptrs`` a CUDA int64 tensor of device pointers
    to column-major matrices (float64, or float32 for mode "fp32"),
    ``orders`` the host list of orders, ``n_dev`` and ``lda_dev`` CUDA int32
    tensors, ``info`` an optional CUDA int32 tensor of the batch size.
    Asynchronous on the current stream; returns ``work``."""
    import torch
    batch = len(orders)
    lib = load()
    o = make_opts(**opts)
    m = _batched_mode(mode)
    h_n = _int_array(orders)
    need = int(lib.batched_spd_inverse_workspace_bytes(batch, h_n, m, ctypes.byref(o)))
    if batch and need == 0:
        raise ValueError("invalid orders (0 <= n <= 2048) or no device")
    dev = ptrs.device
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    rc = lib.batched_spd_inverse(batch, h_n, n_dev.data_ptr(), ptrs.data_ptr(), lda_dev.data_ptr(),
                                 m, work.data_ptr(), need, _stream_ptr(dev),
                                 ctypes.byref(o), info.data_ptr() if info is not None else None)
    if rc != 0:
        raise SpdInverseError(f"batched_spd_inverse returned {rc}")
    return work


def batched_spd_inverse(mats, **opts):
    """Full symmetric inverses of a list of square CUDA tensors, all float64
    (mode "fp64") or all float32 (mode "fp32"); the lower triangle of each is
    read; computed in one batched launch.  Raises NotPositiveDefinite for the
    first matrix whose INFO is positive."""
    import torch
    if not mats:
        return []
    dev = mats[0].device
    dtype = mats[0].dtype
    if dtype not in (torch.float64, torch.float32) or any(m.dtype != dtype for m in mats):
        raise TypeError("expected CUDA tensors, all float64 or all float32")
    mode = "fp64" if dtype == torch.float64 else "fp32"
    esize = 8 if mode == "fp64" else 4
    orders = [int(m.shape[0]) for m in mats]
    sizes = [max(1, n) * max(1, n) for n in orders]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    buf = torch.empty(int(offs[-1]), dtype=dtype, device=dev)
    for m, n, off in zip(mats, orders, offs[:-1]):
        if n:
            # column-major storage of m: its lower triangle is m's lower triangle
            buf[int(off):int(off) + n * n].view(n, n).copy_(m.t())
    base = buf.data_ptr()
    ptrs = torch.tensor([base + esize * int(o) for o in offs[:-1]], dtype=torch.int64, device=dev)
    n_dev = torch.tensor(orders, dtype=torch.int32, device=dev)
    lda_dev = torch.tensor([max(1, n) for n in orders], dtype=torch.int32, device=dev)
    info = torch.zeros(len(mats), dtype=torch.int32, device=dev)
    opts.setdefault("fill_upper", 1)
    batched_spd_inverse_(ptrs, orders, n_dev, lda_dev, mode=mode, info=info, **opts)
    inf = info.cpu().numpy()
    bad = np.nonzero(inf != 0)[0]
    if len(bad):
        k = int(bad[0])
        if inf[k] > 0:
            raise NotPositiveDefinite(int(inf[k]))
        raise SpdInverseError(f"matrix {k}: INFO {int(inf[k])}")
    out = []
    for n, off in zip(orders, offs[:-1]):
        out.append(buf[int(off):int(off) + n * n].view(n, n).t() if n else
                   torch.empty((0, 0), dtype=dtype, device=dev))
    return out


def backward_workspace_bytes(n: int) -> int:
    return int(load().spd_inverse_backward_workspace_bytes(int(n)))


def spd_inverse_backward(x, g, *, work=None, out=None):
    """Gradient of L = sum(g * A^{-1}) with respect to a symmetric A:
    -X sym(g) X, X = A^{-1} (full symmetric n x n CUDA float64, e.g. the
    output of ``spd_inverse``), g any n x n CUDA float64 tensor.  Returns the
    full symmetric gradient (or writes it into ``out``).

    Row-major tensors are passed as column-major buffers of their transposes:
    X is symmetric, sym(g^T) = sym(g) and the result is symmetric, so the
    storage order does not matter."""
    import torch
    for name, v in (("x", x), ("g", g)):
        if v.dtype != torch.float64 or not v.is_cuda or v.dim() != 2:
            raise TypeError(f"{name}: expected a 2-D CUDA float64 tensor")
    n = x.shape[0]
    if x.shape != (n, n) or g.shape != (n, n):
        raise ValueError("x and g must be n x n")
    xc, gc = x.contiguous(), g.contiguous()
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=x.device)
    elif out.shape != (n, n) or not out.is_contiguous() or out.dtype != torch.float64:
        raise ValueError("out must be a contiguous n x n float64 tensor")
    if n == 0:
        return out
    lib = load()
    need = int(lib.spd_inverse_backward_workspace_bytes(n))
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=x.device)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    rc = lib.spd_inverse_backward(n, xc.data_ptr(), n, gc.data_ptr(), n, out.data_ptr(), n,
                                  work.data_ptr(), need, _stream_ptr(x.device))
    if rc != 0:
        raise SpdInverseError(f"spd_inverse_backward returned {rc}")
    return out


def batched_backward_workspace_bytes(orders) -> int:
    return int(load().batched_spd_inverse_backward_workspace_bytes(len(orders),
                                                                   _int_array(orders)))


def batched_spd_inverse_backward_(orders, n_dev, px, ldx, pg, ldg, pout, ldo, work):
    """Low-level batched backward: CUDA int64 tensors of device pointers (px,
    pg, pout: column-major float64 matrices), CUDA int32 tensors of orders
    and leading dimensions, the host list of orders and a workspace of at
    least ``batched_backward_workspace_bytes(orders)`` bytes.  Asynchronous
    on the current stream."""
    lib = load()
    need = int(lib.batched_spd_inverse_backward_workspace_bytes(len(orders), _int_array(orders)))
    if work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    rc = lib.batched_spd_inverse_backward(len(orders), _int_array(orders), n_dev.data_ptr(),
                                          px.data_ptr(), ldx.data_ptr(), pg.data_ptr(),
                                          ldg.data_ptr(), pout.data_ptr(), ldo.data_ptr(),
                                          work.data_ptr(), need, _stream_ptr(work.device))
    if rc != 0:
        raise SpdInverseError(f"batched_spd_inverse_backward returned {rc}")


def batched_spd_inverse_backward(xs, gs, *, work=None, out=None):
    """Gradients -X_i sym(g_i) X_i for lists of square CUDA float64 tensors
    (X_i symmetric, e.g. outputs of ``spd_inverse``; g_i any), computed in one
    persistent launch.  Returns a list of full symmetric gradients (written
    into the tensors of ``out`` when given, contiguous n_i x n_i).  Row-major
    buffers are passed as column-major ones of the transposes, as in
    ``spd_inverse_backward``."""
    import torch
    if len(xs) != len(gs):
        raise ValueError("xs and gs differ in length")
    if not xs:
        return []
    dev = xs[0].device
    orders = []
    for x, g in zip(xs, gs):
        n = x.shape[0]
        if x.dtype != torch.float64 or g.dtype != torch.float64 or not x.is_cuda or not g.is_cuda:
            raise TypeError("expected CUDA float64 tensors")
        if x.shape != (n, n) or g.shape != (n, n):
            raise ValueError("each x and g must be n x n")
        orders.append(int(n))
    xc = [x.contiguous() for x in xs]
    gc = [g.contiguous() for g in gs]
    if out is None:
        out = [torch.empty((n, n), dtype=torch.float64, device=dev) for n in orders]
    elif len(out) != len(xs) or any(o.shape != (n, n) or not o.is_contiguous()
                                    for o, n in zip(out, orders)):
        raise ValueError("out must hold contiguous n_i x n_i tensors")
    lib = load()
    h_n = _int_array(orders)
    need = int(lib.batched_spd_inverse_backward_workspace_bytes(len(orders), h_n))
    if need == 0:
        raise ValueError("invalid orders (0 <= n <= 2048)")
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=dev)
    elif work.numel() * work.element_size() < need:
        raise ValueError(f"workspace too small: need {need} bytes")
    ptr = lambda ts: torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)  # noqa: E731
    ld = torch.tensor([max(1, n) for n in orders], dtype=torch.int32, device=dev)
    n_dev = torch.tensor(orders, dtype=torch.int32, device=dev)
    px, pg, po = ptr(xc), ptr(gc), ptr(out)
    rc = lib.batched_spd_inverse_backward(len(orders), h_n, n_dev.data_ptr(), px.data_ptr(),
                                          ld.data_ptr(), pg.data_ptr(), ld.data_ptr(),
                                          po.data_ptr(), ld.data_ptr(), work.data_ptr(), need,
                                          _stream_ptr(dev))
    if rc != 0:
        raise SpdInverseError(f"batched_spd_inverse_backward returned {rc}")
    # (the pointer tables may be freed now: torch reuses their memory only for
    # work ordered after this launch on the stream)
    return out


def _tuning_dict(t) -> dict:
    return {f: getattr(t, f) for f, _ in _lib.Tuning._fields_}


def autotune(n: int, reps: int = 3) -> dict:
    """Times the FP64 form's schedules at order n on the current device (a
    synthetic SPD matrix, coordinate descent over workgroups per CU, products
    per device task and the row parts of split products) and makes the
    fastest the library's choice for that tile count.  Returns the choice,
    its time and the built-in choice's time."""
    import torch
    t = _lib.Tuning()
    rc = load().spdinv_autotune(int(n), int(reps), _stream_ptr(torch.cuda.current_device()),
                                ctypes.byref(t))
    if rc != 0:
        raise SpdInverseError(f"spdinv_autotune returned {rc}")
    return _tuning_dict(t)


def autotune_batched(orders, mode: str = "fp64", reps: int = 3) -> dict:
    """Times the batched form's schedules for a batch of these orders (on
    synthetic SPD matrices) and makes the fastest the library's choice for
    batches with the same number of matrices of each tile count."""
    import torch
    t = _lib.Tuning()
    rc = load().spdinv_autotune_batched(len(orders), _int_array(orders), _batched_mode(mode),
                                        int(reps),
                                        _stream_ptr(torch.cuda.current_device()), ctypes.byref(t))
    if rc != 0:
        raise SpdInverseError(f"spdinv_autotune_batched returned {rc}")
    return _tuning_dict(t)


def tuning_save(path: str) -> None:
    if load().spdinv_tuning_save(path.encode()) != 0:
        raise OSError(f"cannot write the tuning file {path}")


def tuning_load(path: str) -> None:
    if load().spdinv_tuning_load(path.encode()) != 0:
        raise OSError(f"cannot read the tuning file {path}")


def tuning_clear() -> None:
    load().spdinv_tuning_clear()


def _autograd_function():
    import torch

    class SpdInverse(torch.autograd.Function):
        """A -> A^{-1} for symmetric positive definite A (lower triangle read),
        with the gradient taken over symmetric matrices: dL/dA =
        -A^{-1} sym(dL/dA^{-1}) A^{-1}.  Both directions run in the HIP
        library; with a leading batch dimension each direction is one batched
        launch (batched_spd_inverse, batched_spd_inverse_backward)."""

        @staticmethod
        def forward(ctx, a):
            if a.dim() == 2:
                x = spd_inverse(a)
            else:
                x = torch.stack(batched_spd_inverse(list(a)))
            ctx.save_for_backward(x)
            return x

        @staticmethod
        def backward(ctx, gx):
            (x,) = ctx.saved_tensors
            if x.dim() == 2:
                return spd_inverse_backward(x, gx)
            out = torch.empty_like(x)
            batched_spd_inverse_backward(list(x), list(gx), out=list(out))
            return out

    return SpdInverse


_SPD_FN = None


def __getattr__(name):
    # the autograd Function class is created on first use (torch is imported lazily)
    global _SPD_FN
    if name == "SpdInverse":
        if _SPD_FN is None:
            _SPD_FN = _autograd_function()
        return _SPD_FN
    raise AttributeError(name)


def spd_inverse_ad(a):
    """Differentiable A^{-1} (see ``SpdInverse``)."""
    return __getattr__("SpdInverse").apply(a)


def plan_stats(t: int, **opts) -> dict:
    o = make_opts(**opts)
    st = _lib.PlanStats()
    if load().spdinv_plan_stats_get(int(t), ctypes.byref(o), ctypes.byref(st)) != 0:
        raise ValueError("invalid tile count")
    return {"tasks": st.tasks, "edges": st.edges,
            "count": {TASK_NAMES[k]: st.count[k] for k in range(len(TASK_NAMES))},
            "cp_step": list(st.cp_step), "cp_unpipelined": st.cp_unpipelined,
            "cp_plan": st.cp_plan}


def plan_export(t: int, workers: int = 1, steps: int = 7, rhs_tiles: int = 0, **opts) -> dict:
    """The plan as numpy arrays: tasks (ntasks x 8 int32), succ, step, idx,
    order, and links (nlinks x 2 int32: the further operand pairs of chained
    product tasks).  ``steps``: 7 the SPD inverse, 1 the Cholesky factor
    only, 6 the inverse from a given factor, 9 the solve (factor, then the
    substitutions over ``rhs_tiles`` tile columns), 8 the solve with a given
    factor."""
    lib = load()
    o = make_opts(**opts)
    nt, ns, nl = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    if lib.spdinv_plan_export_steps(int(steps), int(rhs_tiles), int(t), ctypes.byref(o),
                                    int(workers), None, None, None, None, None,
                                    ctypes.byref(nt), ctypes.byref(ns), None,
                                    ctypes.byref(nl)) != 0:
        raise ValueError("invalid tile count or steps")
    tasks = np.zeros((nt.value, 8), dtype=np.int32)
    succ = np.zeros(max(ns.value, 1), dtype=np.int32)
    step = np.zeros(nt.value, dtype=np.int32)
    idx = np.zeros(nt.value, dtype=np.int32)
    order = np.zeros(nt.value, dtype=np.int32)
    links = np.zeros(max(nl.value, 2), dtype=np.int32)
    p = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    lib.spdinv_plan_export_steps(int(steps), int(rhs_tiles), int(t), ctypes.byref(o),
                                 int(workers), p(tasks), p(succ), p(step), p(idx), p(order), None,
                                 None, p(links), None)
    return {"tasks": tasks, "succ": succ[:ns.value], "step": step, "idx": idx, "order": order,
            "links": links[:nl.value].reshape(-1, 2), "t": int(t), "T": t * (t + 1) // 2}


def batch_template_export(t: int, mode: str = "fp64", **opts) -> dict:
    """The batched form's task list for a matrix of t tiles per side:
    tasks (ntask x 8 int32; position 0 the copy-in task, the last the
    copy-out task), succ (positions) and links (nlinks x 2)."""
    lib = load()
    o = make_opts(**opts)
    nt, ns, nl = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
    m = _batched_mode(mode)
    if lib.spdinv_batch_template_export(int(t), m, ctypes.byref(o), None, None, None,
                                        ctypes.byref(nt), ctypes.byref(ns), ctypes.byref(nl)):
        raise ValueError("invalid tile count, mode or options")
    tasks = np.zeros((nt.value, 8), dtype=np.int32)
    succ = np.zeros(max(ns.value, 1), dtype=np.int32)
    links = np.zeros((max(nl.value, 1), 2), dtype=np.int32)
    p = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    lib.spdinv_batch_template_export(int(t), m, ctypes.byref(o), p(tasks), p(succ), p(links),
                                     None, None, None)
    return {"tasks": tasks, "succ": succ[:ns.value], "links": links[:nl.value], "t": int(t)}


def batch_plan_export(orders, mode: str = "fp64", workers: int = 512, **opts) -> dict:
    """The batched form's dispatch list for these orders: disp (tickets, each
    (matrix << 12) | position) and mat (batch x 4 int32: template tile count,
    first counter, first pool tile, 0)."""
    lib = load()
    o = make_opts(**opts)
    h_n = _int_array(orders)
    m = _batched_mode(mode)
    nt = lib.spdinv_batch_plan_export(len(orders), h_n, m, ctypes.byref(o), int(workers), None,
                                      None)
    if nt < 0:
        raise ValueError("invalid orders, mode or options")
    disp = np.zeros(nt, dtype=np.int32)
    mat = np.zeros((len(orders), 4), dtype=np.int32)
    p = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    lib.spdinv_batch_plan_export(len(orders), h_n, m, ctypes.byref(o), int(workers), p(disp),
                                 p(mat))
    return {"disp": disp, "mat": mat}


def trace(work, n: int, **opts) -> np.ndarray:
    """Per-task trace left in ``work`` by a call with trace=1:
    int64 rows (worker, claim, start, end), ticks of the 100 MHz device clock,
    indexed by task (plan order)."""
    lib = load()
    o = make_opts(**opts)
    t = -(-int(n) // 128)
    # the paper's tasks, two barriers and the further row parts of split
    # products (at most 3 each, for at most 2t products)
    nt = plan_stats(t, **{k: v for k, v in opts.items()
                          if k in ("renamed", "loop_order", "pipelined", "trtri_first")})["tasks"]
    nt += 2 + 6 * t
    buf = np.zeros((nt, 4), dtype=np.int64)
    import torch
    torch.cuda.synchronize()
    got = lib.spdinv_trace_copy(work.data_ptr(), int(n), ctypes.byref(o),
                                buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nt)
    if got < 0:
        raise SpdInverseError("no trace available")
    return buf[:got]
