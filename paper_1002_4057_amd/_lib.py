"""ctypes binding of ``libspdinv.so`` (argument marshalling only).

Every function here forwards to the C-ABI declared in ``include/spdinv.h``;
the arithmetic runs in the library's HIP kernels.  Loading fails loudly when
the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspdinv.so")

SPDINV_FP64 = 0
SPDINV_FP32 = 1
SPDINV_MIXED_FP32 = 2
SPDINV_MIXED_BF16 = 3

ERR_WORKSPACE = 1
ERR_HIP = 2
ERR_TIMEOUT = 3
ERR_UNSUPPORTED = 4

NOALLOC_MAX_N = 2048

TASK_NAMES = ["NOP", "SYRK1", "POTRF", "GEMM1", "TRSM1", "TRTRI", "TRMM2L", "GEMM2", "TRSM2R",
              "TRMM3", "LAUUM", "GEMM3", "SYRK3", "GEMMS", "TRSMS", "TADD"]


class Opts(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("pipelined", ctypes.c_int), ("renamed", ctypes.c_int),
                ("loop_order", ctypes.c_int), ("trtri_first", ctypes.c_int),
                ("workers", ctypes.c_int), ("fill_upper", ctypes.c_int), ("trace", ctypes.c_int),
                ("max_refine", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("chain", ctypes.c_int), ("per_cu", ctypes.c_int), ("no_split", ctypes.c_int),
                ("parts", ctypes.c_int), ("rename_tiles", ctypes.c_int),
                ("tree_levels", ctypes.c_int), ("batch_group", ctypes.c_int),
                ("correction64", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int), ("status", ctypes.c_int), ("nb", ctypes.c_int),
                ("tiles", ctypes.c_int), ("tasks", ctypes.c_longlong),
                ("critical_path", ctypes.c_int), ("workers", ctypes.c_int),
                ("refine_iters", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("resid_fro_rel", ctypes.c_double), ("resid0_fro_rel", ctypes.c_double),
                ("resid_last_rel", ctypes.c_double), ("converged", ctypes.c_int),
                ("predicted", ctypes.c_int), ("low_corrections", ctypes.c_int),
                ("resid0_probe_rel", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("per_cu", ctypes.c_int), ("chain", ctypes.c_int),
                ("parts", ctypes.c_int), ("batch_group", ctypes.c_int), ("ms", ctypes.c_double),
                ("ms_default", ctypes.c_double), ("candidates", ctypes.c_int)]


class PlanStats(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_longlong), ("edges", ctypes.c_longlong),
                ("count", ctypes.c_longlong * 16), ("cp_step", ctypes.c_int * 3),
                ("cp_unpipelined", ctypes.c_int), ("cp_plan", ctypes.c_int)]


class LibraryNotBuilt(RuntimeError):
    pass


_lib = None


def load():
    """Loads the HIP library (raises LibraryNotBuilt when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryNotBuilt(
            f"{LIB_PATH} is missing: build it with `python -m paper_1002_4057_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    lib.spdinv_default_opts.argtypes = [P(Opts)]
    lib.spdinv_default_opts.restype = None
    lib.spd_inverse_workspace_bytes.argtypes = [i, i, P(Opts)]
    lib.spd_inverse_workspace_bytes.restype = sz
    lib.spd_inverse.argtypes = [i, vp, i, i, vp, sz, vp, P(Opts), vp, P(Report)]
    lib.spd_inverse.restype = i
    for name in ("spd_cholesky", "spd_inverse_from_factor"):
        fn = getattr(lib, name)
        fn.argtypes = [i, vp, i, vp, sz, vp, P(Opts), vp, P(Report)]
        fn.restype = i
    for name in ("spd_solve", "spd_solve_from_factor"):
        fn = getattr(lib, name)
        fn.argtypes = [i, i, vp, i, vp, i, vp, sz, vp, P(Opts), vp, P(Report)]
        fn.restype = i
    lib.spd_solve_workspace_bytes.argtypes = [i, i, P(Opts)]
    lib.spd_solve_workspace_bytes.restype = sz
    lib.spdinv_release_plans.argtypes = []
    lib.spdinv_release_plans.restype = None
    lib.spdinv_plan_stats_get.argtypes = [i, P(Opts), P(PlanStats)]
    lib.spdinv_plan_stats_get.restype = i
    i32p = P(ctypes.c_int32)
    lib.spdinv_plan_export.argtypes = [i, P(Opts), i, i32p, i32p, i32p, i32p, i32p,
                                       P(ctypes.c_longlong), P(ctypes.c_longlong), i32p,
                                       P(ctypes.c_longlong)]
    lib.spdinv_plan_export.restype = i
    lib.spdinv_plan_export_steps.argtypes = [i, i] + lib.spdinv_plan_export.argtypes
    lib.spdinv_plan_export_steps.restype = i
    lib.spdinv_trace_copy.argtypes = [vp, i, P(Opts), P(ctypes.c_int64), ctypes.c_longlong]
    lib.spdinv_trace_copy.restype = ctypes.c_longlong
    lib.spdinv_kernel_timer.argtypes = [i]
    lib.spdinv_kernel_timer.restype = i
    lib.spdinv_kernel_timer_read.argtypes = [P(ctypes.c_longlong)]
    lib.spdinv_kernel_timer_read.restype = ctypes.c_double
    ip = P(ctypes.c_int)
    lib.batched_spd_inverse_workspace_bytes.argtypes = [i, ip, i, P(Opts)]
    lib.batched_spd_inverse_workspace_bytes.restype = sz
    lib.batched_spd_inverse.argtypes = [i, ip, vp, vp, vp, i, vp, sz, vp, P(Opts), vp]
    lib.batched_spd_inverse.restype = i
    lib.spd_inverse_backward_workspace_bytes.argtypes = [i]
    lib.spd_inverse_backward_workspace_bytes.restype = sz
    lib.spd_inverse_backward.argtypes = [i, vp, i, vp, i, vp, i, vp, sz, vp]
    lib.spd_inverse_backward.restype = i
    ll = ctypes.c_longlong
    lib.spdinv_batch_template_export.argtypes = [i, i, P(Opts), i32p, i32p, i32p, P(ll), P(ll),
                                                 P(ll)]
    lib.spdinv_batch_template_export.restype = i
    lib.spdinv_batch_plan_export.argtypes = [i, ip, i, P(Opts), i, i32p, i32p]
    lib.spdinv_batch_plan_export.restype = ll
    lib.batched_spd_inverse_backward_workspace_bytes.argtypes = [i, ip]
    lib.batched_spd_inverse_backward_workspace_bytes.restype = sz
    lib.batched_spd_inverse_backward.argtypes = [i, ip, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.batched_spd_inverse_backward.restype = i
    lib.spdinv_autotune.argtypes = [i, i, vp, P(Tuning)]
    lib.spdinv_autotune.restype = i
    lib.spdinv_autotune_batched.argtypes = [i, ip, i, i, vp, P(Tuning)]
    lib.spdinv_autotune_batched.restype = i
    lib.spdinv_tuning_clear.argtypes = []
    lib.spdinv_tuning_clear.restype = i
    lib.spdinv_tuning_save.argtypes = [ctypes.c_char_p]
    lib.spdinv_tuning_save.restype = i
    lib.spdinv_tuning_load.argtypes = [ctypes.c_char_p]
    lib.spdinv_tuning_load.restype = i
    lib.spd_inverse_noalloc.argtypes = [i, vp, i, vp, P(Opts), vp]
    lib.spd_inverse_noalloc.restype = i
    lib.spdinv_version.argtypes = []
    lib.spdinv_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_opts(**kw) -> Opts:
    o = Opts()
    load().spdinv_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o
