"""TEST INFRASTRUCTURE: the narrow-slice FP64x2 GEMM (BF16/FP16 slices with
exact FP32 level sums) written out step by step.

Plain numpy in float64 (round-to-nearest-even, one rounding per operation,
numpy never contracts a*b+c).  Only tests, the smoke check and the benchmark's
CPU-baseline leg may use it.  It shares no code with the HIP path.

The method carries the bfloat16 cascade of Sec. 6.2 ("FP32 in terms of
bfloat16": a few bfloat16 splits, products accumulated in FP32 so the bins
need no separate accumulation) to FP64x2, with every split of the same width
and the product set of Sec. 6.1 (equal-width splits: only the t(t+1)/2
leading products are formed).  The INT8 form (Sec. 6.2, "FP64x2 in terms of
INT8": 14-15 splits, 105-120 products, 32-bit integer accumulation) is the
same computation with slices held in int8 and level sums in INT32; only the
chunk of the inner dimension can differ.  Steps, with w the slice width in
bits and s the number of slices:

1. Sigma and T (Sec. 3.4, Appendix A, as in the cascade): one power of two
   per row of A and per column of B, 2^e with e the frexp exponent of the
   largest |fl(hi + lo)| of that row/column, so every scaled entry
   x' = (hi + lo) 2^-e lies in (-1, 1).  A zero row gives e = 0.
2. Slices: with grid u_t = 2^-((t+1)w - 1), slice t of x' is the running
   remainder rounded to a multiple of u_t by (r + K_t) - K_t,
   K_t = 3 * 2^(52 - (t+1)w); the remainder is carried as an unevaluated
   FP64 pair renormalised by TwoSum after each slice.  a_t = d_t / u_t is an
   integer with |a_t| <= 2^(w-1), exact in BF16 (w <= 9), FP16 (w <= 12) or
   INT8 (w <= 7).
   Slices after s are dropped.
3. Level sums: S_L = sum over i + j = L of A_i B_j (integer matrices), for
   L = 0 .. s-1 only (the triangle of Sec. 6.1).  They are exact integers;
   here they are formed with float64 products, exact because every partial
   sum is an integer below 2^53.  (The device forms the same integers on
   BF16/FP16 matrix cores with FP32 accumulation, flushed to FP64 before any
   FP32 partial sum could exceed 2^24; the blocking does not change the
   integers, so the oracle does not model it.)
4. Level groups: G_g = sum over L in {3g, 3g+1, 3g+2}, L < s, of
   S_L 2^(w(3g+2-L)) -- exact while
   k * s * 2^(2w-2) * (2^(2w) + 2^w + 1) <= 2^53 (for INT8 also
   k * s * 2^(2w-2) <= 2^31 - 1); the inner dimension is cut into
   consecutive chunks of at most ``chunk_limit`` indices otherwise, each
   chunk computed and added to C in turn.
5. Combine: V = sum_g G_g W_g with W_g = 2^(2 - (3g+4)w), accumulated in
   FP64x2 from the last (least significant) group to group 0 with the
   FP64x2 + FP64 addition; both words scaled by 2^(e_i + f_j); C added last
   with the accurate FP64x2 addition (Sec. 3.6 order, C last as in the
   cascade).

Readings where the paper is silent (each also listed in the design notes):
the exponent comes from fl(hi + lo) rather than hi; slices are
round-to-nearest on a fixed grid with the remainder renormalised after each
slice; the level-group size is three; chunks of the inner dimension are
added to C one by one.
"""
from __future__ import annotations

import numpy as np

from .cascade import dd_add, dd_add_d, two_sum

# largest slice magnitude each format holds exactly: every integer up to
# 2^8 (BF16, 8 significant bits), 2^11 (FP16), 127 (INT8)
FORMAT_MAX = {"bf16": 2 ** 8, "f16": 2 ** 11, "i8": 127}
FORMAT_BITS = {"bf16": 8, "f16": 11}  # significant bits of the floating-point formats
# Levels per FP64 group: three is the most for which a group stays an exact
# FP64 integer at the default widths over inner dimensions of interest.  A
# group of g levels at w = 8, s = 14 is exact for k s 2^14 2^(8(g-1)) below
# about 2^53: some 596,000 inner indices for g = 3, but only about 2,300 for
# g = 4 (a 4096-deep product would then need two chunks).
GROUP = 3


# ---------------------------------------------------------------- parameters
def check_params(w: int, s: int, fmt: str = "bf16"):
    """Raise ValueError unless (w, s) can run on the device: slices
    (|a| <= 2^(w-1)) exact in ``fmt``; for BF16/FP16 every level's FP32
    partial sums exact over at least one 16-deep matrix-core step
    (16 * s * 2^(2w-2) <= 2^24).  INT8 sums in INT32 over a whole chunk."""
    if fmt not in FORMAT_MAX:
        raise ValueError("fmt must be 'bf16', 'f16' or 'i8'")
    if not (2 <= w and 2 ** (w - 1) <= FORMAT_MAX[fmt]):
        raise ValueError("slice width out of range for the format")
    if not (1 <= s <= 16):
        raise ValueError("slice count must be in [1, 16]")
    if fmt != "i8" and 16 * s * 2 ** (2 * w - 2) > 2 ** 24:
        raise ValueError("FP32 level sums would not be exact for one 16-deep step")


def flush_depths(w: int, s: int):
    """For level L (L + 1 products), the largest power-of-two block of inner
    indices kb_L >= 16 with kb_L (L+1) 2^(2w-2) <= 2^24: the FP32 partial sums
    of that level stay exact integers over kb_L inner indices."""
    out = []
    for L in range(s):
        kb = 16
        while 2 * kb * (L + 1) * 2 ** (2 * w - 2) <= 2 ** 24:
            kb *= 2
        out.append(kb)
    return out


def chunk_limit(w: int, s: int, fmt: str = "bf16"):
    """Largest number of inner indices per chunk allowed by the exactness
    bounds alone: every level group sum an exact FP64 integer,
    k s 2^(2w-2) (2^2w + 2^w + 1) <= 2^53, and for INT8 also every level sum
    an INT32, k s 2^(2w-2) <= 2^31 - 1.  Chunk c covers inner indices
    [c * limit, (c + 1) * limit)."""
    per = s * 2 ** (2 * w - 2) * (2 ** (2 * w) + 2 ** w + 1)
    lim = 2 ** 53 // per
    if fmt == "i8":
        lim = min(lim, (2 ** 31 - 1) // (s * 2 ** (2 * w - 2)))
    return lim


def n_products(s: int) -> int:
    return s * (s + 1) // 2


# ------------------------------------------------------------ Sigma, T, split
def slice_exponents(hi, lo, axis):
    """e with max |fl(hi + lo)| along ``axis`` in [2^(e-1), 2^e); zero -> 0."""
    hi = np.asarray(hi, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    if hi.shape[axis] == 0:
        return np.zeros(hi.shape[1 - axis], dtype=np.int32)
    with np.errstate(invalid="ignore", over="ignore"):
        mx = np.max(np.abs(hi + lo), axis=axis)   # NaN if the row holds one
        _, e = np.frexp(mx)                        # frexp(Inf or NaN) gives 0
    return np.where(np.isfinite(mx), e, 0).astype(np.int32)


def split_slices(hi, lo, e, axis, w, s):
    """Slices a_0 .. a_{s-1} (integer-valued float64 arrays) of (hi + lo) 2^-e,
    e broadcast along ``axis`` (axis=1: one e per row; axis=0: per column),
    and the dropped remainder as an unevaluated pair (r, rho)."""
    shift = -np.asarray(e, dtype=np.int64)
    shift = shift[:, None] if axis == 1 else shift[None, :]
    with np.errstate(invalid="ignore", over="ignore"):
        r, rho = two_sum(np.ldexp(np.asarray(hi, dtype=np.float64), shift),
                         np.ldexp(np.asarray(lo, dtype=np.float64), shift))
        out = []
        for t in range(s):
            K = 3.0 * 2.0 ** (52 - (t + 1) * w)
            d = (r + K) - K
            out.append(d * 2.0 ** ((t + 1) * w - 1))
            r, rho = two_sum(r - d, rho)
    return out, (r, rho)


# ----------------------------------------------------------------- products
def level_sums(As, Bs, s):
    """S_L = sum_{i+j=L} A_i B_j for L < s (exact integers as float64)."""
    out = []
    for L in range(s):
        acc = None
        for i in range(L + 1):
            p = As[i] @ Bs[L - i]
            acc = p if acc is None else acc + p
        out.append(acc)
    return out


def group_sums(S, w):
    """G_g = sum_{L in group g} S_L 2^(w (3g+2-L)) (exact)."""
    s = len(S)
    out = []
    for g in range((s + GROUP - 1) // GROUP):
        acc = None
        for L in range(GROUP * g, min(s, GROUP * g + GROUP)):
            term = S[L] * 2.0 ** (w * (GROUP * g + GROUP - 1 - L))
            acc = term if acc is None else acc + term
        out.append(acc)
    return out


def group_weight(g, w):
    """W_g = 2^(2 - (3g+4) w): the value of one unit of G_g."""
    return 2.0 ** (2 - (GROUP * g + GROUP + 1) * w)


def combine_groups(G, w):
    """sum_g G_g W_g in FP64x2, least significant group first."""
    acc_h = np.zeros_like(G[0])
    acc_l = np.zeros_like(G[0])
    for g in range(len(G) - 1, -1, -1):
        acc_h, acc_l = dd_add_d(acc_h, acc_l, G[g] * group_weight(g, w))
    return acc_h, acc_l


# -------------------------------------------------------------------- GEMM
def slices_gemm(A, B, C=None, *, w=8, s=14, fmt="bf16", return_parts=False):
    """C + A B by the slices variant; A (m×k), B (k×n), C (m×n) as (hi, lo).

    Returns ``(hi, lo)``; with ``return_parts`` also a dict with the
    exponents, the slices, the level sums and group sums of the last chunk.
    """
    check_params(w, s, fmt)
    Ahi, Alo = (np.asarray(x, dtype=np.float64) for x in A)
    Bhi, Blo = (np.asarray(x, dtype=np.float64) for x in B)
    m, k = Ahi.shape
    n = Bhi.shape[1]
    if C is None:
        Rh, Rl = np.zeros((m, n)), np.zeros((m, n))
    else:
        Rh, Rl = (np.array(x, dtype=np.float64) for x in C)
    if k == 0 or m == 0 or n == 0:
        return (Rh, Rl, {}) if return_parts else (Rh, Rl)
    e = slice_exponents(Ahi, Alo, axis=1)
    f = slice_exponents(Bhi, Blo, axis=0)
    As, _ = split_slices(Ahi, Alo, e, 1, w, s)
    Bs, _ = split_slices(Bhi, Blo, f, 0, w, s)
    shift = e.astype(np.int64)[:, None] + f.astype(np.int64)[None, :]
    step = chunk_limit(w, s, fmt)
    parts = {"e": e, "f": f, "A": As, "B": Bs}
    with np.errstate(invalid="ignore", over="ignore"):
        for p0 in range(0, k, step):
            p1 = min(k, p0 + step)
            S = level_sums([a[:, p0:p1] for a in As], [b[p0:p1, :] for b in Bs], s)
            G = group_sums(S, w)
            vh, vl = combine_groups(G, w)
            vh = np.ldexp(vh, shift)
            vl = np.ldexp(vl, shift)
            Rh, Rl = dd_add(Rh, Rl, vh, vl)
            parts.update({"S": S, "G": G})
    return (Rh, Rl, parts) if return_parts else (Rh, Rl)


def slices_gemm_entries(A, B, C, I, J, *, w=8, s=14, fmt="bf16"):
    """Entries (I[t], J[t]) of C + A B by the slices variant (same steps as
    ``slices_gemm`` on the needed rows of A and columns of B)."""
    check_params(w, s, fmt)
    Ahi, Alo = (np.asarray(x, dtype=np.float64) for x in A)
    Bhi, Blo = (np.asarray(x, dtype=np.float64) for x in B)
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    k = Ahi.shape[1]
    rows = Ahi[I], Alo[I]
    cols = Bhi[:, J], Blo[:, J]
    e = slice_exponents(*rows, axis=1)
    f = slice_exponents(*cols, axis=0)
    Rh = np.asarray(C[0], dtype=np.float64)[I, J].copy()
    Rl = np.asarray(C[1], dtype=np.float64)[I, J].copy()
    if k == 0:
        return Rh, Rl
    As, _ = split_slices(*rows, e, 1, w, s)     # len(I) x k
    Bs, _ = split_slices(*cols, f, 0, w, s)     # k x len(J)
    step = chunk_limit(w, s, fmt)
    shift = e.astype(np.int64) + f.astype(np.int64)
    with np.errstate(invalid="ignore", over="ignore"):
        for p0 in range(0, k, step):
            p1 = min(k, p0 + step)
            S = []
            for L in range(s):
                acc = np.zeros(len(I))
                for i in range(L + 1):
                    acc = acc + np.einsum("tp,pt->t", As[i][:, p0:p1], Bs[L - i][p0:p1, :])
                S.append(acc)
            G = group_sums(S, w)
            vh, vl = combine_groups(G, w)
            Rh, Rl = dd_add(Rh, Rl, np.ldexp(vh, shift), np.ldexp(vl, shift))
    return Rh, Rl
