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


# ---- IEEE binary64 operations defined by rounding the exact rational result
def rn(x: Fraction) -> float:
    """Round a rational to the nearest double, ties to even (CPython's
    int / int true division is correctly rounded)."""
    return float(x)


def add_rn(a: float, b: float) -> float:
    return rn(Fraction(a) + Fraction(b))


def sub_rn(a: float, b: float) -> float:
    return rn(Fraction(a) - Fraction(b))


def two_sum_exact(a: float, b: float):
    """The error-free sum by its definition: s = RN(a + b) and the exact
    remainder a + b - s (a double whenever no overflow occurs)."""
    s = add_rn(a, b)
    e = Fraction(a) + Fraction(b) - Fraction(s)
    assert rn(e) == e
    return s, rn(e)


def quick_two_sum_ops(a: float, b: float):
    """Dekker's fast two-sum as its three rounded operations:
    s = RN(a + b), e = RN(b - RN(s - a))."""
    s = add_rn(a, b)
    return s, sub_rn(b, sub_rn(s, a))


def dd_add_d_ops(h: float, l: float, y: float):
    """FP64x2 (h, l) plus an FP64 y: error-free sum of the high parts, the
    low part added with one rounding, then a fast two-sum."""
    s, e = two_sum_exact(h, y)
    return quick_two_sum_ops(s, add_rn(e, l))
