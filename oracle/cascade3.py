"""TEST INFRASTRUCTURE: the cascade for FP64x3 (triple-word) operands written
out step by step, in plain numpy (float64, one rounding per operation).

The paper only names this case (Sec. 6.2, FP64x3 in terms of FP64: six
FP64 splits).  The steps follow the FP64x2 cascade of Sec. 3 with six
digits instead of four:

1. Split widths (c0..c4) for a rank-kc block: the largest widths (in total,
   then in order) for which every bin 0..4 is exact (``widths3``): bin L
   sums kc (L+1) products A_i' B_j' (i + j = L) whose digits are at most 3
   in units of their level (three words each contribute at most 1), on the
   finest grid of that bin; the sum must stay below 2^53 grid steps.
2. Sigma and T: 2^e per row of A (column of B), e the frexp exponent of the
   largest |x0| (the leading word), as for FP64x2.
3. Split: each word scaled by 2^-e is cut as in Appendix A into five digits
   on the grids 2^(1-c_t) and a remainder; digits of the three words are
   added level by level (exact for levels 0..4: at most three multiples of
   the level grid below 3 in magnitude), the remainders rounded
   ((d5(x0) + d5(x1)) + d5(x2)).  Planes are pre-weighted,
   A_t' = 2^-D_(t-1) D_t.
4. Products per rank-kc block: bins L = 0..4 are sum_(i+j=L) A_i' B_j'
   (exact); the tail bin is sum_i A_i' U_(5-i)' with the suffix sums
   U_t' = B_t' + U_(t+1)' of B's planes (U_5' = B_5', each addition
   rounded once, from the last plane up to U_0') -- the analogue of B4',
   B5', B6' (Sec. 3.4).
5. The six bins are summed exactly and rounded to a triple word
   (``td_round``), the rank-kc results accumulated the same way (the exact
   sum of the two triple words, rounded), Sigma and T applied (exact), C
   added last.

``td_round`` is the plain definition of triple-word rounding: the exact
sum S of the terms (rational arithmetic), w0 = RN(S), w1 = RN(S - w0),
w2 = RN(S - w0 - w1).  It stands for any faithful triple-word summation:
the device's error-free sequence of TwoSums is held to it within a bound.

Readings where the paper is silent are listed in the design notes (FP64x3
section).
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np

from .cascade import exponents, two_sum

D = 53
NDIG = 6            # digits per word: five fixed-point, one remainder
DIGIT_MAX = 3.0     # |D_t| in units of its level, three words


@functools.lru_cache(maxsize=None)
def widths3(kc: int):
    """(c0..c4) for rank-kc blocks: the exactness rule of step 1, largest
    total D4 first, then lexicographically largest.  (The rule only gets
    easier as widths shrink, so for each c0..c3 the largest feasible c4 is
    the one to keep.)"""
    if kc < 1:
        raise ValueError("kc must be >= 1")
    best = None
    rng = range(26, 13, -1)
    for c0 in rng:
        for c1 in rng:
            for c2 in rng:
                for c3 in rng:
                    for c4 in rng:
                        c = (c0, c1, c2, c3, c4)
                        if exact_bins_ok(c, kc):
                            key = (sum(c), c)
                            if best is None or key > best:
                                best = key
                            break
    return best[1]


def exact_bins_ok(c, kc):
    """Step 1's rule: for every bin L <= 4 the largest possible sum, in steps
    of the bin's finest grid, is below 2^53 (all quantities are sums of a few
    powers of two times 9, exact in float64)."""
    Dc = [sum(c[:t + 1]) for t in range(5)]   # D_t = c_0 + ... + c_t
    Dm = [0] + Dc[:-1]                        # D_(t-1), D_(-1) = 0
    for L in range(5):
        pairs = [(i, L - i) for i in range(L + 1)]
        # A_i' is a multiple of 2^(1 - D_i) of magnitude <= 3 * 2^-D_(i-1)
        fine = min(2 - Dc[i] - Dc[j] for i, j in pairs)
        total = 0.0
        for i, j in pairs:
            total += math.ldexp(DIGIT_MAX * DIGIT_MAX * kc, -Dm[i] - Dm[j] - fine)
        if total >= 2.0 ** 53:
            return False
    return True


def split_word(v, c):
    """Appendix A on scaled FP64 values v: [d0..d4, d5]."""
    v = np.array(v, dtype=np.float64, copy=True)
    out = []
    for ct in c:
        K = 2.0 ** (D - ct) + 2.0 ** (D - 1 - ct)
        d = (v + K) - K
        v = (v - d) * (2.0 ** ct)
        out.append(d)
    out.append(v)
    return out


def split3(words, e, axis, c):
    """Pre-weighted planes [A_0'..A_5'] of the FP64x3 operand ``words`` =
    (x0, x1, x2) scaled by 2^-e (e per row for axis=1, per column for axis=0),
    and the three scaled words."""
    shift = -np.asarray(e, dtype=np.int64)
    shift = shift[:, None] if axis == 1 else shift[None, :]
    scaled = [np.ldexp(np.asarray(w, dtype=np.float64), shift) for w in words]
    digs = [split_word(w, c) for w in scaled]
    Dl = [digs[0][t] + digs[1][t] + digs[2][t] for t in range(5)]
    Dl.append((digs[0][5] + digs[1][5]) + digs[2][5])
    Dc = np.cumsum(c)
    weights = [1.0] + [2.0 ** -int(Dc[t]) for t in range(5)]
    return [Dl[t] * weights[t] for t in range(6)], scaled


def suffix_planes(Bp):
    """U_5' = B_5' and U_t' = B_t' + U_(t+1)' for t = 4 .. 0, each addition
    rounded once (from the last plane up)."""
    U = [None] * 6
    U[5] = Bp[5]
    for t in range(4, -1, -1):
        U[t] = Bp[t] + U[t + 1]
    return U


def _rn_scaled(num: int, exp: int) -> float:
    """RN(num * 2^exp) for an integer num.  float(num) is the correctly
    rounded (to nearest, ties to even) conversion; scaling by 2^exp is exact
    unless the result leaves the normal range, where the rational value is
    rounded directly instead."""
    if num == 0:
        return 0.0
    if abs(num).bit_length() > 1000:
        return float(Fraction(num) * Fraction(2) ** exp)
    try:
        w = math.ldexp(float(num), exp)
    except OverflowError:
        w = math.inf
    if abs(w) < 2.0 ** -1021 or math.isinf(w):
        return float(Fraction(num) * Fraction(2) ** exp)
    return w


def _round3(num: int, exp: int):
    """(w0, w1, w2) with w0 = RN(S), w1 = RN(S - w0), w2 = RN(S - w0 - w1)
    for S = num * 2^exp."""
    out = []
    for _ in range(3):
        w = _rn_scaled(num, exp)
        out.append(w)
        if w != 0.0:
            mant, ex = math.frexp(w)                 # w = mant 2^ex, a multiple of 2^exp
            sh = ex - 53 - exp
            wi = int(math.ldexp(mant, 53))
            num -= wi << sh if sh >= 0 else wi >> -sh
    return tuple(out)


def td_round(terms):
    """The exact sum of ``terms`` (arrays of one shape) rounded to a triple
    word, entry by entry.  Every double is an integer times 2^-1074, so the
    sum is taken exactly as an integer over the smallest exponent present.
    An entry with a non-finite term gives NaN words."""
    arrs = [np.asarray(t, dtype=np.float64) for t in terms]
    shape = arrs[0].shape
    flat = [a.reshape(-1) for a in arrs]
    out = np.empty((3, flat[0].size))
    for q in range(flat[0].size):
        vals = [float(a[q]) for a in flat]
        if not all(math.isfinite(v) for v in vals):
            out[:, q] = np.nan
            continue
        parts = []
        for v in vals:
            if v != 0.0:
                mant, ex = math.frexp(v)                 # v = mant 2^ex, 0.5 <= |mant| < 1
                parts.append((int(math.ldexp(mant, 53)), ex - 53))
        if not parts:
            out[:, q] = 0.0
            continue
        e0 = min(ex for _, ex in parts)
        num = sum(mant << (ex - e0) for mant, ex in parts)
        out[:, q] = _round3(num, e0)
    return tuple(out[w].reshape(shape) for w in range(3))


def td_add(x, y):
    """x + y for triple words x = (x0, x1, x2), y likewise: the exact sum
    rounded to a triple word."""
    return td_round([x[0], x[1], x[2], y[0], y[1], y[2]])


def bins3_block(Ap, Bp, U, p0, p1):
    """Bins 0..4 and the tail bin for inner indices [p0, p1)."""
    a = [x[:, p0:p1] for x in Ap]
    b = [x[p0:p1, :] for x in Bp]
    u = [x[p0:p1, :] for x in U]
    bins = []
    for L in range(5):
        s = a[0] @ b[L]
        for i in range(1, L + 1):
            s = s + a[i] @ b[L - i]
        bins.append(s)
    tail = a[0] @ u[5]
    for i in range(1, 6):
        tail = tail + a[i] @ u[5 - i]
    bins.append(tail)
    return bins


def cascade3_gemm(A, B, C=None, *, kc=256, return_parts=False):
    """C + A B for FP64x3 operands given as (x0, x1, x2) word triples."""
    A = [np.asarray(x, dtype=np.float64) for x in A]
    B = [np.asarray(x, dtype=np.float64) for x in B]
    m, k = A[0].shape
    n = B[0].shape[1]
    Cw = [np.zeros((m, n)) for _ in range(3)] if C is None else [np.array(x, dtype=np.float64) for x in C]
    if k == 0 or m == 0 or n == 0:
        return tuple(Cw)
    kce = min(int(kc), k)
    c = widths3(kce)
    e = exponents(A[0], axis=1)
    f = exponents(B[0], axis=0)
    Ap, _ = split3(A, e, 1, c)
    Bp, _ = split3(B, f, 0, c)
    U = suffix_planes(Bp)
    acc = (np.zeros((m, n)), np.zeros((m, n)), np.zeros((m, n)))
    blocks = []
    for p0 in range(0, k, kce):
        p1 = min(k, p0 + kce)
        bins = bins3_block(Ap, Bp, U, p0, p1)
        blk = td_round(bins)
        acc = td_add(acc, blk)
        if return_parts:
            blocks.append(bins)
    shift = e.astype(np.int64)[:, None] + f.astype(np.int64)[None, :]
    acc = tuple(np.ldexp(x, shift) for x in acc)
    R = td_add(tuple(Cw), acc)
    if return_parts:
        return R, {"c": c, "kc": kce, "A": Ap, "B": Bp, "U": U, "e": e, "f": f, "bins": blocks}
    return R


def eps3(kc: int) -> float:
    """2^-(D4 + 53): the unit of the last digit (the FP64x3 analogue of the
    2^-(D2 + 53) of Sec. 3.2)."""
    return 2.0 ** -(sum(widths3(kc)) + D)


def digits_bound_ok(kc: int) -> bool:
    return exact_bins_ok(widths3(kc), kc)


def log2_ceil(x: int) -> int:
    return int(math.ceil(math.log2(x))) if x > 1 else 0
