"""C-ABI surface (CPU only, no compute): the built library loads, exports
every function declared in include/spdinv.h, and rejects invalid arguments
on the host before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_1002_4057_amd as spd
from paper_1002_4057_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "spdinv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(spd\w+|spdinv_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_loads_and_reports_version():
    lib = _lib.load()
    assert b"gfx950" in lib.spdinv_version()


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = declared_functions()
    assert {"spd_inverse", "spd_inverse_workspace_bytes", "spdinv_plan_stats_get"} <= set(names)
    for name in names:
        assert hasattr(lib, name), f"{name} declared in spdinv.h but not exported"


def test_library_links_no_oracle_code():
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"oracle_" not in data


def test_workspace_bytes():
    assert spd.workspace_bytes(0) == 0
    t = 4
    pool = (3 * t * (t + 1) // 2 + 2 * t) * 128 * 128 * 8
    assert spd.workspace_bytes(512) >= pool
    assert spd.workspace_bytes(513) > spd.workspace_bytes(512)
    assert spd.workspace_bytes(512, trace=1) > spd.workspace_bytes(512)


@pytest.mark.parametrize("args,code", [
    ((-1, 1, 1, 0), -1),     # n < 0
    ((4, 0, 4, 0), -2),      # null A
    ((4, 1, 3, 0), -3),      # lda < n
    ((4, 1, 4, 7), -4),      # unknown mode
])
def test_invalid_arguments_rejected_on_host(args, code):
    lib = _lib.load()
    n, a, lda, mode = args
    rc = lib.spd_inverse(n, a, lda, mode, None, 0, None, None, None, None)
    assert rc == code


def test_bad_options_rejected():
    lib = _lib.load()
    o = spd.make_opts(nb=96)
    assert lib.spd_inverse(4, 1, 4, 0, 1, 1 << 30, None, ctypes.byref(o), None, None) == -8
    o = spd.make_opts(loop_order=5)
    assert lib.spd_inverse(4, 1, 4, 0, 1, 1 << 30, None, ctypes.byref(o), None, None) == -8


def test_too_small_workspace_rejected():
    lib = _lib.load()
    assert lib.spd_inverse(512, 1, 512, 0, 1, 16, None, None, None, None) == _lib.ERR_WORKSPACE
    assert lib.spd_inverse(512, 1, 512, 0, None, 0, None, None, None, None) == -5


@pytest.mark.parametrize("args,code", [
    ((-1, 1, 1, 1, 1, 1, 1), -1),   # n < 0
    ((4, 0, 4, 1, 4, 1, 4), -2),    # null X
    ((4, 1, 3, 1, 4, 1, 4), -3),    # ldx < n
    ((4, 1, 4, 0, 4, 1, 4), -4),    # null G
    ((4, 1, 4, 1, 2, 1, 4), -5),    # ldg < n
    ((4, 1, 4, 1, 4, 0, 4), -6),    # null gradA
    ((4, 1, 4, 1, 4, 1, 1), -7),    # ldga < n
])
def test_backward_invalid_arguments_rejected_on_host(args, code):
    lib = _lib.load()
    n, x, ldx, g, ldg, ga, ldga = args
    assert lib.spd_inverse_backward(n, x, ldx, g, ldg, ga, ldga, 1, 1 << 40, None) == code


def test_backward_workspace():
    lib = _lib.load()
    assert lib.spd_inverse_backward_workspace_bytes(0) == 0
    assert lib.spd_inverse_backward_workspace_bytes(129) == 3 * 4 * 128 * 128 * 8
    assert lib.spd_inverse_backward(0, None, 1, None, 1, None, 1, None, 0, None) == 0
    assert lib.spd_inverse_backward(8, 1, 8, 1, 8, 1, 8, None, 0, None) == -8
    assert lib.spd_inverse_backward(8, 1, 8, 1, 8, 1, 8, 1, 16, None) == _lib.ERR_WORKSPACE


def test_batched_invalid_arguments_rejected_on_host():
    lib = _lib.load()
    n = (ctypes.c_int * 2)(4, 5)
    assert lib.batched_spd_inverse(-1, n, 1, 1, 1, 0, 1, 1 << 40, None, None, None) == -1
    assert lib.batched_spd_inverse(0, None, None, None, None, 0, None, 0, None, None, None) == 0
    assert lib.batched_spd_inverse(2, None, 1, 1, 1, 0, 1, 1 << 40, None, None, None) == -2
    assert lib.batched_spd_inverse(2, n, None, 1, 1, 0, 1, 1 << 40, None, None, None) == -3
    assert lib.batched_spd_inverse(2, n, 1, None, 1, 0, 1, 1 << 40, None, None, None) == -4
    assert lib.batched_spd_inverse(2, n, 1, 1, None, 0, 1, 1 << 40, None, None, None) == -5
    assert lib.batched_spd_inverse(2, n, 1, 1, 1, 2, 1, 1 << 40, None, None, None) == -6
    o = spd.make_opts(nb=64)
    assert lib.batched_spd_inverse(2, n, 1, 1, 1, 0, 1, 1 << 40, None, ctypes.byref(o), None) == -10
    o = spd.make_opts(renamed=0)     # the FP32 tile tasks take the renamed plan only
    assert lib.batched_spd_inverse(2, n, 1, 1, 1, _lib.SPDINV_FP32, 1, 1 << 40, None,
                                   ctypes.byref(o), None) == -10
    big = (ctypes.c_int * 2)(4, 2049)
    assert lib.batched_spd_inverse(2, big, 1, 1, 1, 0, 1, 1 << 40, None, None, None) == -2
    assert lib.batched_spd_inverse(2, n, 1, 1, 1, 0, 1, 16, None, None, None) == _lib.ERR_WORKSPACE


def test_batched_workspace_bytes():
    # with three matrices and 512 simulated workers all run at once: every
    # matrix above one tile has a pool slot of its own, 3T + 2t tiles
    orders = [100, 129, 256, 300]
    b64 = spd.batched_workspace_bytes(orders)
    b32 = spd.batched_workspace_bytes(orders, mode="fp32")
    pools = sum(3 * t * (t + 1) // 2 + 2 * t for t in (2, 2, 3)) * 128 * 128
    assert b64 >= pools * 8 and b32 >= pools * 4 and b32 < b64
    assert spd.batched_workspace_bytes([2049]) == 0
    # the list-scheduled DAG on one simulated worker: the two matrices of two
    # tiles share one slot
    one = spd.batched_workspace_bytes(orders, workers=1, batch_group=-2)
    assert one < b64 and one >= (3 * 3 + 4 + 3 * 6 + 6) * 128 * 128 * 8
    # one workgroup per matrix: a pool of the largest tile count per workgroup
    seq = spd.batched_workspace_bytes(orders, workers=2, batch_group=-1)
    assert 2 * (3 * 6 + 6) * 128 * 128 * 8 <= seq < 2 * (3 * 6 + 6) * 128 * 128 * 8 + (1 << 20)


def test_mixed_mode_host_checks():
    lib = _lib.load()
    o = spd.make_opts(renamed=0)
    assert lib.spd_inverse(4, 1, 4, _lib.SPDINV_MIXED_FP32, 1, 1 << 30, None, ctypes.byref(o),
                           None, None) == -8
    # the FP32 form runs the renamed plan only and checks its workspace
    assert lib.spd_inverse(4, 1, 4, _lib.SPDINV_FP32, 1, 1 << 30, None, ctypes.byref(o), None,
                           None) == -8
    assert lib.spd_inverse(512, 1, 512, _lib.SPDINV_FP32, 1, 16, None, None, None,
                           None) == _lib.ERR_WORKSPACE
    assert 0 < spd.workspace_bytes(1000, mode="fp32") < spd.workspace_bytes(1000)
    assert lib.spd_inverse(4, 1, 4, 9, 1, 1 << 30, None, None, None, None) == -4
    assert lib.spd_inverse(4, 1, 4, _lib.SPDINV_MIXED_BF16, 1, 1 << 30, None, ctypes.byref(o),
                           None, None) == -8
    assert spd.workspace_bytes(1000, mode="mixed_bf16") == spd.workspace_bytes(1000,
                                                                               mode="mixed_fp32")
    assert spd.workspace_bytes(1000, mode="mixed_fp32") > spd.workspace_bytes(1000)
    assert lib.spd_inverse(512, 1, 512, _lib.SPDINV_MIXED_FP32, 1, 16, None, None, None,
                           None) == _lib.ERR_WORKSPACE


def test_every_source_is_built():
    from paper_1002_4057_amd import build
    csrc = os.path.join(ROOT, "paper_1002_4057_amd", "csrc")
    srcs = {f for f in os.listdir(csrc) if f.endswith((".hip", ".cpp"))}
    assert srcs == set(build.SOURCES)


def test_batched_backward_arguments_rejected_on_host():
    lib = _lib.load()
    n = (ctypes.c_int * 2)(4, 300)
    # 4 t^2 tiles per matrix (t = 1 and 3) and the counters
    tiles = (4 * 1 + 4 * 9) * 128 * 128 * 8
    assert tiles <= lib.batched_spd_inverse_backward_workspace_bytes(2, n) < tiles + 4096
    assert lib.batched_spd_inverse_backward_workspace_bytes(1, (ctypes.c_int * 1)(2049)) == 0
    args = [1, 1, 1, 1, 1, 1, 1, 1, 1, 1 << 40, None]
    assert lib.batched_spd_inverse_backward(-1, n, *args) == -1
    assert lib.batched_spd_inverse_backward(0, None, *args) == 0
    assert lib.batched_spd_inverse_backward(2, None, *args) == -2
    for pos in range(1, 9):   # d_n, d_X, d_ldx, d_G, d_ldg, d_gradA, d_ldga, work
        a = list(args)
        a[pos - 1] = None
        assert lib.batched_spd_inverse_backward(2, n, *a) == -(pos + 2)
    a = list(args)
    a[9] = 16
    assert lib.batched_spd_inverse_backward(2, n, *a) == _lib.ERR_WORKSPACE


@pytest.mark.parametrize("opts,mode,code", [
    (dict(correction64=2), 2, -8),          # not 0 or 1
    (dict(tree_levels=1), 1, -8),           # the FP32 form runs the sequential chains
    (dict(tree_levels=1), 2, -8),           # so do the mixed forms
    (dict(tree_levels=3), 0, -8),           # at most 2 levels
    (dict(rename_tiles=10), 3, -8),         # partial renaming is FP64 only
])
def test_options_of_the_forms_rejected_on_host(opts, mode, code):
    """Rejected by the host checks, before any device call."""
    lib = _lib.load()
    o = spd.make_opts(**opts)
    assert lib.spd_inverse(4, 1, 4, mode, 1, 1 << 30, None, ctypes.byref(o), None, None) == code


def test_noalloc_rejects_the_tree_and_the_trace():
    lib = _lib.load()
    for opts in (dict(tree_levels=1), dict(trace=1)):
        o = spd.make_opts(**opts)
        assert lib.spd_inverse_noalloc(4, 1, 4, None, ctypes.byref(o), None) == -5
