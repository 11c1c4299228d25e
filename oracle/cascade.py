"""TEST INFRASTRUCTURE: the cascaded FP64x2 GEMM written out step by step.

Plain, slow numpy (float64, round-to-nearest-even, one rounding per
operation; numpy never contracts a*b+c).  Only tests, the smoke check and the
benchmark's CPU-baseline leg may use it.  It shares no code with the HIP path.

Steps, in the paper's order and notation:

1. Split widths (c0, c1, c2) from the rank-kc inner size (Sec. 3.3, the four
   exactness constraints on bins 0-2, with ceil(log2 kc)); c3 is a full FP64.
   D0 = c0, D1 = c0+c1, D2 = c0+c1+c2, sigma_1 = 2^-D0, sigma_2 = 2^-D1,
   sigma_3 = 2^-D2 (Sec. 3.2).
2. Sigma and T (Sec. 3.3-3.4, Appendix A): one power of two per row of A and
   per column of B, 2^e with e the frexp exponent of the largest |hi| in that
   row/column, so the scaled entries lie in (-1, 1).  A zero row gives e = 0.
3. Split (Appendix A): hi and lo are scaled by 2^-e and cut separately; each
   digit is (v + K) - K with K = 2^(53-c) + 2^(52-c), the remainder is
   multiplied by 2^c; the fourth digit keeps what is left.  Digits of hi and
   lo are added level by level.
4. The ten products of eq. (Gemm10) per rank-kc update, with pre-weighted
   planes A_t' = sigma_t A_t and B_t' = sigma_t B_t:
     bin 0   = A0' B0'
     bin 1   = A0' B1' + A1' B0'
     bin 2   = A0' B2' + A1' B1' + A2' B0'
     bin 3-6 = A0' B3' + A1' B4' + A2' B5' + A3' B6'
   where B4' = sigma_2 B4 = B2' + B3', B5' = sigma_1 B5 = B1' + B4' and
   B6 = B0 + sigma_1 B1 + sigma_2 B2 + sigma_3 B3 (Sec. 3.4, the definitions
   of B4, B5, B6).  Bins 0-2 are exact in FP64; bin 3-6 is rounded.
5. Across bins in FP64x2, least significant first (Sec. 3.3; Sec. 3.6, the
   expression for fl_casc): bin0 + (bin1 + (bin2 + fl(bin 3-6))); the
   rank-kc results are accumulated in FP64x2 (Sec. 4.2, Fig. gemmrankk).
6. Apply Sigma and T (Sec. 4.2) and add C last.  (Option: Sigma and T per
   rank-kc panel, each panel's result scaled before it is accumulated; the
   paper packs and splits one kc panel at a time, Sec. 4.3.)  (Option: a
   power-of-two diagonal balancing F applied first, A B = (A F)(F^-1 B),
   Sec. 6; see ``balance_exponents``.)
7. Cancellation flags (Sec. 3.7, Sec. 4.4): an entry is flagged when bin 0
   of a rank-kc block is zero while a lower bin of that block is not.

Readings where the paper is silent (each also listed in the design notes):
B4', B5' and B6' are each rounded once to FP64 (B6' = RN(hi*2^-f + lo*2^-f));
the fourth digit is RN(d3(hi) + d3(lo)); Sigma and T are global over the whole
k; the kc-blocks are consecutive runs of kc inner indices starting at 0.
"""
from __future__ import annotations

import numpy as np

D = 53


# ---------------------------------------------------------------- parameters
def split_widths(kc: int):
    """(c0, c1, c2) for rank-kc updates: 2c0+L<=53, c0+c1+L+1<=53, 2c1+L+2<=53,
    c0+c2+L+2<=53 with L = ceil(log2 kc) (Sec. 3.3)."""
    if kc < 1:
        raise ValueError("kc must be >= 1")
    L = (int(kc) - 1).bit_length()
    c0 = (D - L) // 2
    c1 = min(D - L - 1 - c0, (D - L - 2) // 2)
    c2 = D - L - 2 - c0
    return c0, c1, c2


def sigmas(c):
    """(sigma_1, sigma_2, sigma_3) = (2^-D0, 2^-D1, 2^-D2) (Sec. 3.2)."""
    c0, c1, c2 = c
    return 2.0 ** -c0, 2.0 ** -(c0 + c1), 2.0 ** -(c0 + c1 + c2)


# ------------------------------------------------------------- DD arithmetic
def two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def quick_two_sum(a, b):
    s = a + b
    e = b - (s - a)
    return s, e


def dd_add_d(xh, xl, y):
    """FP64x2 + FP64."""
    s, e = two_sum(xh, y)
    e = e + xl
    return quick_two_sum(s, e)


def dd_add(xh, xl, yh, yl):
    """FP64x2 + FP64x2 (accurate variant: two TwoSums, two renormalisations)."""
    s, e = two_sum(xh, yh)
    t, f = two_sum(xl, yl)
    e = e + t
    s, e = quick_two_sum(s, e)
    e = e + f
    return quick_two_sum(s, e)


# ------------------------------------------------------------ Sigma, T, split
def exponents(hi, axis):
    """e with max |hi| along ``axis`` in [2^(e-1), 2^e); all-zero -> 0."""
    hi = np.asarray(hi, dtype=np.float64)
    if hi.shape[axis] == 0:
        return np.zeros(hi.shape[1 - axis], dtype=np.int32)
    _, e = np.frexp(np.max(np.abs(hi), axis=axis))
    return e.astype(np.int32)


def split_fp64(v, c):
    """Appendix A on FP64 values v (already scaled): returns [d0, d1, d2, d3]."""
    v = np.array(v, dtype=np.float64, copy=True)
    digits = []
    for ct in c:
        K = 2.0 ** (D - ct) + 2.0 ** (D - 1 - ct)
        d = (v + K) - K
        v = (v - d) * (2.0 ** ct)
        digits.append(d)
    digits.append(v)
    return digits


def split_fp64x2(hi, lo, e, axis, c):
    """Digits [d0..d3] of the FP64x2 entries (hi, lo) scaled by 2^-e, with e
    broadcast along ``axis`` (axis=1: one e per row; axis=0: one per column)."""
    shift = -np.asarray(e, dtype=np.int64)
    shift = shift[:, None] if axis == 1 else shift[None, :]
    xh = np.ldexp(np.asarray(hi, dtype=np.float64), shift)
    xl = np.ldexp(np.asarray(lo, dtype=np.float64), shift)
    dh = split_fp64(xh, c)
    dl = split_fp64(xl, c)
    return [dh[t] + dl[t] for t in range(4)], xh, xl


def cascade_A(hi, lo, c):
    """Pre-weighted planes [A0', A1', A2', A3'] and the row exponents of A."""
    e = exponents(hi, axis=1)
    d, _, _ = split_fp64x2(hi, lo, e, 1, c)
    s1, s2, s3 = sigmas(c)
    return [d[0], d[1] * s1, d[2] * s2, d[3] * s3], e


def cascade_B(hi, lo, c):
    """Pre-weighted planes [B0', ..., B6'] and the column exponents of B."""
    f = exponents(hi, axis=0)
    d, yh, yl = split_fp64x2(hi, lo, f, 0, c)
    s1, s2, s3 = sigmas(c)
    B0, B1, B2, B3 = d[0], d[1] * s1, d[2] * s2, d[3] * s3
    B4 = B2 + B3
    B5 = B1 + B4
    B6 = yh + yl
    return [B0, B1, B2, B3, B4, B5, B6], f


# ----------------------------------------------------------------- products
def bins_block(Ap, Bp, p0, p1):
    """Bins 0, 1, 2 and 3-6 of eq. (Gemm10) for inner indices [p0, p1)."""
    a = [x[:, p0:p1] for x in Ap]
    b = [x[p0:p1, :] for x in Bp]
    bin0 = a[0] @ b[0]
    bin1 = a[0] @ b[1] + a[1] @ b[0]
    bin2 = a[0] @ b[2] + a[1] @ b[1] + a[2] @ b[0]
    bin36 = a[0] @ b[3] + a[1] @ b[4] + a[2] @ b[5] + a[3] @ b[6]
    return bin0, bin1, bin2, bin36


def combine_bins(bin0, bin1, bin2, bin36):
    """bin0 + (bin1 + (bin2 + bin36)) in FP64x2 (Sec. 3.6)."""
    s, e = two_sum(bin2, bin36)
    s, e = dd_add_d(s, e, bin1)
    s, e = dd_add_d(s, e, bin0)
    return s, e


def cancellation_flags(blocks):
    """Sec. 3.7 / Sec. 4.4: an entry is at risk of cancellation when a rank-kc
    block's bin 0 (the leading digits' product, exact) is zero while one of
    its lower bins is not.  ``blocks`` is the list of (bin0, bin1, bin2,
    bin36) of every block (``cascade_gemm(..., return_parts=True)["bins"]``).
    For k <= kc this is the paper's check on bin 0; a block whose bins are
    all zero (zero row or column segment) carries no risk and is not
    flagged."""
    flag = None
    for b0, b1, b2, b36 in blocks:
        f = (b0 == 0) & ((b1 != 0) | (b2 != 0) | (b36 != 0))
        flag = f if flag is None else (flag | f)
    return flag


def balance_exponents(Ahi, Bhi):
    """Power-of-two diagonal balancing F (Sec. 6, scaling and balancing:
    A B = (A F)(F^-1 B)).  For inner index p, with e_A(p) the exponent of
    column p of A and e_B(p) that of row p of B (step 2's exponent rule), the
    balancing exponent is g_p = floor((e_B(p) - e_A(p)) / 2): A's column is
    multiplied by 2^g_p and B's row by 2^-g_p, which leaves both near the
    geometric mean of the two maxima."""
    eA = exponents(Ahi, axis=0).astype(np.int64)
    eB = exponents(Bhi, axis=1).astype(np.int64)
    return (eB - eA) // 2


def cascade_gemm(A, B, C=None, *, kc=256, c=None, scaling="global", balance=False, return_parts=False):
    """C + A B by the cascade; A (m×k), B (k×n), C (m×n) as (hi, lo) pairs.

    The rank-kc block is ``min(kc, k)`` and the split widths follow from it,
    unless ``c`` fixes them (the paper's k_C = 256 setting is c = (22, 21, 21)).
    ``scaling="panel"`` takes Sigma and T per rank-kc panel instead (step 2
    applied to each panel A[:, p0:p1], B[p0:p1, :] on its own; the panel's
    FP64x2 result is scaled by its own powers of two before it joins the
    accumulator, and no scaling is left for the end).
    Returns ``(hi, lo)``; with ``return_parts`` also a dict holding the planes,
    exponents and the bins of every rank-kc block.
    """
    if scaling not in ("global", "panel"):
        raise ValueError("scaling must be 'global' or 'panel'")
    if balance:
        # ``balance=True`` first multiplies column p of A by 2^g_p and row p of
        # B by 2^-g_p (``balance_exponents``); the product is unchanged
        # (exactly, barring underflow), the split sees balanced operands
        g = balance_exponents(np.asarray(A[0], dtype=np.float64), np.asarray(B[0], dtype=np.float64))
        A = tuple(np.ldexp(np.asarray(x, dtype=np.float64), g[None, :]) for x in A)
        B = tuple(np.ldexp(np.asarray(x, dtype=np.float64), -g[:, None]) for x in B)
    Ahi, Alo = (np.asarray(x, dtype=np.float64) for x in A)
    Bhi, Blo = (np.asarray(x, dtype=np.float64) for x in B)
    m, k = Ahi.shape
    n = Bhi.shape[1]
    if C is None:
        Chi, Clo = np.zeros((m, n)), np.zeros((m, n))
    else:
        Chi, Clo = (np.array(x, dtype=np.float64) for x in C)
    if k == 0 or m == 0 or n == 0:
        return (Chi, Clo, {}) if return_parts else (Chi, Clo)
    kc_eff = min(int(kc), k)
    c = split_widths(kc_eff) if c is None else tuple(int(v) for v in c)
    if scaling == "panel":
        return _cascade_panels(Ahi, Alo, Bhi, Blo, Chi, Clo, kc_eff, c, return_parts)
    Ap, e = cascade_A(Ahi, Alo, c)
    Bp, f = cascade_B(Bhi, Blo, c)
    acc_h = np.zeros((m, n))
    acc_l = np.zeros((m, n))
    blocks = []
    for p0 in range(0, k, kc_eff):
        p1 = min(k, p0 + kc_eff)
        b = bins_block(Ap, Bp, p0, p1)
        th, tl = combine_bins(*b)
        acc_h, acc_l = dd_add(acc_h, acc_l, th, tl)
        if return_parts:
            blocks.append(b)
    shift = e.astype(np.int64)[:, None] + f.astype(np.int64)[None, :]
    acc_h = np.ldexp(acc_h, shift)
    acc_l = np.ldexp(acc_l, shift)
    Rh, Rl = dd_add(Chi, Clo, acc_h, acc_l)
    if return_parts:
        return Rh, Rl, {"c": c, "kc": kc_eff, "A": Ap, "B": Bp, "e": e, "f": f, "bins": blocks}
    return Rh, Rl


def _cascade_panels(Ahi, Alo, Bhi, Blo, Chi, Clo, kc, c, return_parts):
    """The cascade with Sigma and T of each rank-kc panel (``scaling="panel"``)."""
    m, k = Ahi.shape
    n = Bhi.shape[1]
    acc_h = np.zeros((m, n))
    acc_l = np.zeros((m, n))
    blocks, es, fs = [], [], []
    for p0 in range(0, k, kc):
        p1 = min(k, p0 + kc)
        Ap, e = cascade_A(Ahi[:, p0:p1], Alo[:, p0:p1], c)
        Bp, f = cascade_B(Bhi[p0:p1, :], Blo[p0:p1, :], c)
        b = bins_block(Ap, Bp, 0, p1 - p0)
        th, tl = combine_bins(*b)
        shift = e.astype(np.int64)[:, None] + f.astype(np.int64)[None, :]
        acc_h, acc_l = dd_add(acc_h, acc_l, np.ldexp(th, shift), np.ldexp(tl, shift))
        if return_parts:
            blocks.append(b)
            es.append(e)
            fs.append(f)
    Rh, Rl = dd_add(Chi, Clo, acc_h, acc_l)
    if return_parts:
        return Rh, Rl, {"c": c, "kc": kc, "e": np.array(es), "f": np.array(fs), "bins": blocks}
    return Rh, Rl
