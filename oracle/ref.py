"""TEST INFRASTRUCTURE: ctypes binding of the plain FP64x2 triple-loop GEMM.

``dd_gemm_ref`` computes C := op(A) op(B) + C in double-double arithmetic
(TwoProd by FMA, accurate DD addition, p ascending, C added last): the
FP64x2-arithmetic reference of Sec. 5.2.  Only tests, the smoke check and
the benchmark's CPU-baseline leg use it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        lib.oracle_dd_gemm.argtypes = [i64, i64, i64, ci, ci, vp, vp, i64, vp, vp, i64,
                                       vp, vp, i64, ci]
        lib.oracle_dd_gemm.restype = ci
        lib.oracle_dd_gemm_entries.argtypes = [i64, vp, vp, i64, ci, ci, vp, vp, i64,
                                               vp, vp, i64, vp, vp, i64, vp, vp, ci]
        lib.oracle_dd_gemm_entries.restype = ci
        lib.oracle_max_threads.restype = ci
        lib.oracle_exact_entries.argtypes = [i64, vp, vp, i64, vp, vp, i64, vp, vp, i64, vp, vp, i64,
                                             vp, vp, vp, vp, ci]
        lib.oracle_exact_entries.restype = ci
        lib.oracle_dd_add_vec.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        lib.oracle_dd_add_vec.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_f(a):
    return np.asfortranarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def dd_gemm_ref(A, B, C=None, *, transa=False, transb=False, threads=0):
    """Return ``(hi, lo, threads_used)`` of op(A) op(B) + C.

    ``A``, ``B``, ``C`` are ``(hi, lo)`` pairs of 2-D float64 arrays as stored
    (before op).  ``C=None`` means zero.
    """
    Ahi, Alo = _as_f(A[0]), _as_f(A[1])
    Bhi, Blo = _as_f(B[0]), _as_f(B[1])
    m = Ahi.shape[1] if transa else Ahi.shape[0]
    k = Ahi.shape[0] if transa else Ahi.shape[1]
    n = Bhi.shape[0] if transb else Bhi.shape[1]
    kb = Bhi.shape[1] if transb else Bhi.shape[0]
    assert kb == k, "inner dimensions differ"
    if C is None:
        Chi = np.zeros((m, n), order="F")
        Clo = np.zeros((m, n), order="F")
    else:
        Chi, Clo = np.array(C[0], dtype=np.float64, order="F"), np.array(C[1], dtype=np.float64, order="F")
        assert Chi.shape == (m, n)
    lda, ldb, ldc = max(1, Ahi.shape[0]), max(1, Bhi.shape[0]), max(1, m)
    used = _load().oracle_dd_gemm(m, n, k, int(transa), int(transb), _ptr(Ahi), _ptr(Alo), lda,
                                  _ptr(Bhi), _ptr(Blo), ldb, _ptr(Chi), _ptr(Clo), ldc, int(threads))
    return Chi, Clo, int(used)


def dd_gemm_ref_entries(A, B, C, I, J, *, transa=False, transb=False, threads=0):
    """Entries ``(I[t], J[t])`` of op(A) op(B) + C; returns ``(hi, lo, threads_used)``."""
    Ahi, Alo = _as_f(A[0]), _as_f(A[1])
    Bhi, Blo = _as_f(B[0]), _as_f(B[1])
    Chi, Clo = _as_f(C[0]), _as_f(C[1])
    k = Ahi.shape[0] if transa else Ahi.shape[1]
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out_hi = np.empty(I.shape[0])
    out_lo = np.empty(I.shape[0])
    used = _load().oracle_dd_gemm_entries(
        I.shape[0], _ptr(I), _ptr(J), k, int(transa), int(transb),
        _ptr(Ahi), _ptr(Alo), max(1, Ahi.shape[0]), _ptr(Bhi), _ptr(Blo), max(1, Bhi.shape[0]),
        _ptr(Chi), _ptr(Clo), max(1, Chi.shape[0]), _ptr(out_hi), _ptr(out_lo), int(threads))
    return out_hi, out_lo, int(used)


def exact_entries(A, B, C, I, J, R, *, threads=0):
    """Exact value of entries (I[t], J[t]) of A B + C (FP64x2 operands as
    stored, no transposes) and the exact difference R - exact for computed
    results ``R = (hi, lo)`` at those entries, both rounded to double.
    Returns ``(exact, err)``."""
    Ahi, Alo = _as_f(A[0]), _as_f(A[1])
    Bhi, Blo = _as_f(B[0]), _as_f(B[1])
    Chi, Clo = _as_f(C[0]), _as_f(C[1])
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    Rh = np.ascontiguousarray(R[0], dtype=np.float64)
    Rl = np.ascontiguousarray(R[1], dtype=np.float64)
    exact = np.empty(I.shape[0])
    err = np.empty(I.shape[0])
    st = _load().oracle_exact_entries(
        I.shape[0], _ptr(I), _ptr(J), Ahi.shape[1], _ptr(Ahi), _ptr(Alo), max(1, Ahi.shape[0]),
        _ptr(Bhi), _ptr(Blo), max(1, Bhi.shape[0]), _ptr(Chi), _ptr(Clo), max(1, Chi.shape[0]),
        _ptr(Rh), _ptr(Rl), _ptr(exact), _ptr(err), int(threads))
    if st < 0:
        raise RuntimeError("expansion too long (exponent range of the inputs too wide)")
    return exact, err


def dd_add_ref(x, y):
    """Entry-wise accurate FP64x2 sum of two ``(hi, lo)`` pairs of arrays of
    equal shape: ``(hi, lo)`` of x + y, the addition the triple loop
    accumulates with (TwoSum of both words, two renormalisations)."""
    xh, xl = (np.ascontiguousarray(v, dtype=np.float64) for v in x)
    yh, yl = (np.ascontiguousarray(v, dtype=np.float64) for v in y)
    if not (xh.shape == xl.shape == yh.shape == yl.shape):
        raise ValueError("dd_add_ref: shapes differ")
    zh, zl = np.empty_like(xh), np.empty_like(xh)
    _load().oracle_dd_add_vec(xh.size, _ptr(xh), _ptr(xl), _ptr(yh), _ptr(yl), _ptr(zh), _ptr(zl))
    return zh, zl
