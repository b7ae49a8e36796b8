"""Plain FP64 CPU oracle for the SPD inverse (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never links or calls it,
and it shares no code with the GPU path: the arithmetic lives in
``spd_oracle.c`` (plain loops, natural summation order, IEEE binary64).

Every function takes numpy arrays and follows the three stages of the paper's
Algorithm 1 at tile order b = 1 (Section 2):

* :func:`potrf`   -- stage 1, Cholesky factor L of A = L L^T
* :func:`trtri`   -- stage 2, X = L^{-1}
* :func:`lauum`   -- stage 3, A^{-1} = X^T X (lower triangle)
* :func:`spd_inverse` -- the three stages in sequence
* :func:`inverse_grad` -- -Y S Y with S = (G + G^T)/2, Y = A^{-1}
* :func:`potrs`   -- the solve A X = B with the factor L (substitutions)

Matrices are handled as ordinary (row-major) numpy arrays of the *full*
matrix; the wrapper converts to the column-major lower-triangle convention of
the C code.  Results are returned as new arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_spd.so")
_lib = None


class OracleInfo(RuntimeError):
    """Raised when the matrix is not positive definite (LAPACK-style INFO)."""

    def __init__(self, info: int):
        super().__init__(f"leading minor of order {info} is not positive definite")
        self.info = info


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i = ctypes.c_int
    lib.oracle_potrf.argtypes = [i, dp, i, dp, i]
    lib.oracle_potrf.restype = i
    lib.oracle_trtri.argtypes = [i, dp, i, dp, i]
    lib.oracle_trtri.restype = i
    lib.oracle_lauum.argtypes = [i, dp, i, dp, i]
    lib.oracle_lauum.restype = None
    lib.oracle_spd_inverse.argtypes = [i, dp, i]
    lib.oracle_spd_inverse.restype = i
    lib.oracle_inverse_grad.argtypes = [i, dp, i, dp, i, dp, i]
    lib.oracle_inverse_grad.restype = i
    lib.oracle_potrs.argtypes = [i, i, dp, i, dp, i]
    lib.oracle_potrs.restype = i
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = i
    lib.oracle_set_num_threads.argtypes = [i]
    lib.oracle_set_num_threads.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(_LIB)
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _colmajor(a: np.ndarray) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def set_num_threads(nt: int) -> None:
    _load().oracle_set_num_threads(int(nt))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def potrf(a: np.ndarray) -> np.ndarray:
    """Stage 1: lower Cholesky factor of the lower triangle of ``a``."""
    a = _colmajor(a)
    n = a.shape[0]
    out = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().oracle_potrf(n, _ptr(a), max(1, n), _ptr(out), max(1, n))
    if info:
        raise OracleInfo(info)
    return np.ascontiguousarray(out)


def trtri(l: np.ndarray) -> np.ndarray:
    """Stage 2: inverse of the lower triangle of ``l``."""
    l = _colmajor(l)
    n = l.shape[0]
    out = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().oracle_trtri(n, _ptr(l), max(1, n), _ptr(out), max(1, n))
    if info:
        raise OracleInfo(info)
    return np.ascontiguousarray(out)


def lauum(x: np.ndarray) -> np.ndarray:
    """Stage 3: lower triangle of X^T X for lower triangular X (upper zero)."""
    x = _colmajor(x)
    n = x.shape[0]
    out = np.zeros((n, n), dtype=np.float64, order="F")
    _load().oracle_lauum(n, _ptr(x), max(1, n), _ptr(out), max(1, n))
    return np.ascontiguousarray(np.tril(out))


def potrs(l: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve with the Cholesky factor: X with L L^T X = B (forward, then
    backward substitution; only the lower triangle of ``l`` is read)."""
    l = _colmajor(l)
    n = l.shape[0]
    b2 = np.array(b, dtype=np.float64, order="F", copy=True)
    if b2.ndim == 1:
        b2 = b2.reshape(n, 1, order="F")
    nrhs = b2.shape[1]
    info = _load().oracle_potrs(n, nrhs, _ptr(l), max(1, n), _ptr(b2), max(1, n))
    if info:
        raise OracleInfo(info)
    return np.ascontiguousarray(b2).reshape(np.shape(b))


def spd_inverse_lower(a: np.ndarray) -> np.ndarray:
    """All three stages in place on a copy; returns the column-major buffer.

    The strictly upper triangle of the returned (n x n) array is the input's,
    untouched; the lower triangle holds A^{-1}.
    """
    a = _colmajor(a).copy(order="F")
    n = a.shape[0]
    info = _load().oracle_spd_inverse(n, _ptr(a), max(1, n))
    if info:
        raise OracleInfo(info)
    return np.ascontiguousarray(a)


def spd_inverse(a: np.ndarray) -> np.ndarray:
    """Full symmetric A^{-1} from the lower triangle of ``a``."""
    low = np.tril(spd_inverse_lower(a))
    return low + np.tril(low, -1).T


def inverse_grad(y: np.ndarray, g: np.ndarray) -> np.ndarray:
    """-Y S Y with S = (G + G^T)/2; Y given by its lower triangle."""
    y = _colmajor(y)
    g = _colmajor(g)
    n = y.shape[0]
    out = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().oracle_inverse_grad(n, _ptr(y), max(1, n), _ptr(g), max(1, n),
                                       _ptr(out), max(1, n))
    if info:
        raise RuntimeError("oracle_inverse_grad failed to allocate")
    return np.ascontiguousarray(out)


class _Bound:
    """The module's functions bound to another build of the oracle source.

    Used only by the mutation tests, which compile deliberately broken copies
    of ``spd_oracle.c`` to show that the pins catch them.
    """

    def __init__(self, path: str):
        self._lib_path = path
        self._handle = _bind(path)

    def __getattr__(self, name):
        fn = globals()[name]
        if not callable(fn):
            raise AttributeError(name)

        def call(*args, **kwargs):
            global _lib
            saved = _lib
            _lib = self._handle
            try:
                return fn(*args, **kwargs)
            finally:
                _lib = saved

        return call


def load_variant(path: str) -> "_Bound":
    return _Bound(path)
