"""Exact rational arithmetic helpers for pinning the oracle (tests only)."""
from fractions import Fraction

import numpy as np


def F(x):
    return Fraction(float(x))


def dd_value(hi, lo):
    """Exact value of each FP64x2 entry as an object array of Fractions."""
    hi = np.asarray(hi)
    lo = np.asarray(lo)
    out = np.empty(hi.shape, dtype=object)
    for idx in np.ndindex(hi.shape):
        out[idx] = F(hi[idx]) + F(lo[idx])
    return out


def exact_gemm(A, B, C=None):
    """Exact C + A B for small FP64x2 matrices given as (hi, lo)."""
    a = dd_value(*A)
    b = dd_value(*B)
    m, k = a.shape
    n = b.shape[1]
    out = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            s = Fraction(0)
            for p in range(k):
                s += a[i, p] * b[p, j]
            out[i, j] = s
    if C is not None:
        c = dd_value(*C)
        out = out + c
    return out


def abs_gemm(A, B):
    """(|A||B|)_ij exactly, from the FP64x2 values."""
    a = np.abs(dd_value(*A))
    b = np.abs(dd_value(*B))
    m, k = a.shape
    n = b.shape[1]
    out = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            s = Fraction(0)
            for p in range(k):
                s += a[i, p] * b[p, j]
            out[i, j] = s
    return out
