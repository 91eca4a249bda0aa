"""Oracle for the GEMM hot path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_1908_09606_amd``) and never imports it.

Contents
  gemm()            plain binary64 product, the definition of section 2.4 /
                    the CDAG update rule of section 5.1 (``oracle.c``)
  normalised_err()  max_ij |C - C_ref| / D_ij with D = |alpha||A||B| + |beta||C0|
  fp64_bound(k), fp32_bound(k)   the stated error bounds 4k*2^-53, 8k*2^-24
  exact             Fraction brute force for tiny inputs (pins the C code)
  schedule          the paper's I/O model: Theorem 1, Theorem 2, the optimal
                    tile of section 5, eq. optTileShape, grid fitting
                    (section 7.1) and a red-blue pebble simulator
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.oracle_gemm.argtypes = [i64, i64, i64, dbl, vp, i64, vp, i64, dbl, vp, i64, vp, i64,
                                    vp, i64, ctypes.c_int]
        lib.oracle_gemm.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _ptr(a):
    return None if a is None else a.ctypes.data


def gemm(A, B, alpha: float = 1.0, beta: float = 0.0, C0=None, want_bound: bool = True,
         threads: int | None = None):
    """Return (C, D): the binary64 product and the bound matrix D.

    A (m x k) and B (k x n) may be any real dtype; they are widened to
    binary64 exactly.  C0 (m x n) is read only when beta != 0.
    """
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shape mismatch")
    m, k = A.shape
    n = B.shape[1]
    if beta != 0.0:
        C0 = np.ascontiguousarray(C0, dtype=np.float64)
        if C0.shape != (m, n):
            raise ValueError("C0 shape mismatch")
    else:
        C0 = None
    C = np.empty((m, n), dtype=np.float64)
    D = np.empty((m, n), dtype=np.float64) if want_bound else None
    rc = _load().oracle_gemm(m, n, k, float(alpha), _ptr(A), max(k, 1), _ptr(B), max(n, 1),
                             float(beta), _ptr(C0), max(n, 1), _ptr(C), max(n, 1), _ptr(D),
                             max(n, 1), int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("oracle_gemm failed")
    return C, D


def fp64_bound(k: int) -> float:
    """Stated FP64-class bound on the normalised error: 4k * 2^-53."""
    return 4.0 * max(int(k), 1) * 2.0 ** -53


def fp32_bound(k: int) -> float:
    """Stated FP32-class bound on the normalised error: 8k * 2^-24."""
    return 8.0 * max(int(k), 1) * 2.0 ** -24


def normalised_err(C, C_ref, D) -> float:
    """max_ij |C - C_ref| / D_ij.

    Where D_ij == 0 the entry must match exactly (else the error is inf);
    any NaN or Inf in C gives inf.
    """
    C = np.asarray(C, dtype=np.float64)
    C_ref = np.asarray(C_ref, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    if C.shape != C_ref.shape or C.shape != D.shape:
        raise ValueError("shape mismatch")
    if C.size == 0:
        return 0.0
    if not np.all(np.isfinite(C)):
        return float("inf")
    diff = np.abs(C - C_ref)
    zero = D == 0.0
    if np.any(diff[zero] != 0.0):
        return float("inf")
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(zero, 0.0, diff / np.where(zero, 1.0, D))
    return float(r.max())
