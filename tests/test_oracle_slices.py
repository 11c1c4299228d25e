"""Pins of the numpy model of the narrow-slice (BF16/FP16) variant (CPU only).

Against: exact reconstruction of every entry from its slices with rationals,
the slice magnitude bound that makes the FP32 level sums exact, and
representability in the slice format; level sums against integer arithmetic;
results against exact rational C + A B within the truncation bound of the
triangle of Sec. 6.1 (derived in the design notes: at most
(s + 1) 2^-(s w) per inner index relative to the row and column scales, plus
FP64x2 rounding); exact results for integer matrices that fit one slice;
power-of-two row/column equivariance; the FP64x2 oracle's tolerance; the
order of the group sum (least significant group first) on groups where the
two orders round differently; chunk boundaries at multiples of the
exactness limit.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import slices as sl
from oracle.ref import dd_gemm_ref
from paper_2303_04353_amd.inputs import make_problem
from tests.exact import dd_add_d_ops, dd_value, exact_gemm

CONFIGS = [(8, 14), (9, 12), (7, 16), (5, 9), (8, 4), (9, 2)]


def test_params_rules():
    sl.check_params(8, 14)
    sl.check_params(9, 12)
    sl.check_params(9, 16)
    sl.check_params(9, 12, "f16")
    sl.check_params(10, 4, "f16")
    sl.check_params(11, 1, "f16")
    sl.check_params(7, 16, "i8")
    sl.check_params(7, 1, "i8")
    for bad in [(10, 4, "bf16"), (9, 17, "bf16"), (10, 5, "f16"), (12, 1, "f16"), (1, 4, "bf16"),
                (8, 0, "bf16"), (8, 4, "f32"), (8, 16, "i8"), (7, 17, "i8")]:
        with pytest.raises(ValueError):
            sl.check_params(*bad)
    assert [sl.n_products(s) for s in (12, 13, 14)] == [78, 91, 105]


@pytest.mark.parametrize("w,s", [(8, 14), (9, 12), (9, 16), (5, 9)])
def test_flush_depths_are_the_largest_exact_blocks(w, s):
    kb = sl.flush_depths(w, s)
    for L, b in enumerate(kb):
        assert b >= 16 and b & (b - 1) == 0
        assert b * (L + 1) * 2 ** (2 * w - 2) <= 2 ** 24
        assert 2 * b * (L + 1) * 2 ** (2 * w - 2) > 2 ** 24
    if (w, s) == (8, 14):
        assert kb == [1024, 512, 256, 256, 128, 128, 128, 128, 64, 64, 64, 64, 64, 64]


def test_chunk_limit_keeps_group_sums_below_2_53():
    for w, s in CONFIGS:
        c = sl.chunk_limit(w, s)
        assert c > 0
        worst = c * s * 2 ** (2 * w - 2) * (2 ** (2 * w) + 2 ** w + 1)
        assert worst <= 2 ** 53
        # the exactness bound alone decides: one index more breaks it
        assert (c + 1) * s * 2 ** (2 * w - 2) * (2 ** (2 * w) + 2 ** w + 1) > 2 ** 53
    assert sl.chunk_limit(8, 14) > 8192 and sl.chunk_limit(9, 12) > 8192


def _values():
    rng = np.random.default_rng(21)
    hi = list(rng.uniform(-1, 1, 300))
    hi += [0.0, 1.0 - 2.0 ** -53, -(1.0 - 2.0 ** -53), 0.5, -0.5, 2.0 ** -7, 3 * 2.0 ** -9, 2.0 ** -60,
           -2.0 ** -300, 0.75 + 2.0 ** -52, 2.0 ** -8 + 2.0 ** -9, 0.5 + 2.0 ** -8]
    hi += list(rng.uniform(-1, 1, 100) * 2.0 ** rng.integers(-90, 0, 100))
    hi = np.array(hi)
    lo = hi * 2.0 ** -53 * rng.uniform(-1, 1, hi.shape)
    # a few pairs that are not normalised (|lo| larger than half an ulp of hi)
    lo[:5] = hi[:5] * 2.0 ** -30
    return hi, lo


@pytest.mark.parametrize("w,s", CONFIGS)
def test_slices_reconstruct_exactly_and_obey_the_bound(w, s):
    hi, lo = _values()
    H, Lo = hi.reshape(1, -1), lo.reshape(1, -1)
    e = sl.slice_exponents(H, Lo, axis=1)
    slices, (r, rho) = sl.split_slices(H, Lo, e, 1, w, s)
    assert len(slices) == s
    for idx in range(hi.size):
        x = (Fraction(float(hi[idx])) + Fraction(float(lo[idx]))) * Fraction(2) ** -int(e[0])
        assert abs(x) < 1
        total = Fraction(0)
        for t, a in enumerate(slices):
            v = float(a[0, idx])
            assert v == int(v) and abs(v) <= 2 ** (w - 1)
            total += Fraction(int(v)) * Fraction(2) ** -((t + 1) * w - 1)
        rem = Fraction(float(r[0, idx])) + Fraction(float(rho[0, idx]))
        assert total + rem == x                       # nothing lost or invented
        u_last = Fraction(2) ** -(s * w - 1)
        assert abs(rem) <= u_last / 2 * (1 + Fraction(1, 2 ** 40))


@pytest.mark.parametrize("fmt,bits", [("bf16", 8), ("f16", 11)])
def test_slices_fit_the_format(fmt, bits):
    # integers of magnitude <= 2^(w-1) have at most w-1 <= p significant bits
    w = bits + 1
    s = 1 if fmt == "f16" else 4
    if fmt == "f16":
        w = 11   # 16 * 1 * 2^20 <= 2^24
    sl.check_params(w, s, fmt)
    hi, lo = _values()
    e = sl.slice_exponents(hi.reshape(1, -1), lo.reshape(1, -1), axis=1)
    slices, _ = sl.split_slices(hi.reshape(1, -1), lo.reshape(1, -1), e, 1, w, s)
    for a in slices:
        v = np.abs(a).astype(np.int64)
        nz = v[v > 0]
        # significant bits: position of the top bit minus the trailing zeros
        sig = np.array([int(x).bit_length() - ((int(x) & -int(x)).bit_length() - 1) for x in nz])
        assert sig.size == 0 or sig.max() <= bits
        if fmt == "bf16":
            # the top 16 bits of the float32 pattern hold the value exactly
            f32 = a.astype(np.float32)
            assert np.array_equal(f32.view(np.uint32) & 0xFFFF, np.zeros_like(f32.view(np.uint32)))
        else:
            assert np.array_equal(a.astype(np.float16).astype(np.float64), a)


def test_level_sums_match_integer_arithmetic():
    P = make_problem(5, 6, 37, cfg=101)
    w, s = 8, 6
    e = sl.slice_exponents(*P["A"], axis=1)
    f = sl.slice_exponents(*P["B"], axis=0)
    As, _ = sl.split_slices(*P["A"], e, 1, w, s)
    Bs, _ = sl.split_slices(*P["B"], f, 0, w, s)
    S = sl.level_sums(As, Bs, s)
    ai = [[[int(x) for x in row] for row in a] for a in As]
    bi = [[[int(x) for x in row] for row in b] for b in Bs]
    for L in range(s):
        for i in range(5):
            for j in range(6):
                want = 0
                for t in range(L + 1):
                    want += sum(ai[t][i][p] * bi[L - t][p][j] for p in range(37))
                assert S[L][i, j] == want
    G = sl.group_sums(S, w)
    assert len(G) == 2
    for i in range(5):
        for j in range(6):
            assert G[0][i, j] == int(S[0][i, j]) * 2 ** 16 + int(S[1][i, j]) * 2 ** 8 + int(S[2][i, j])


def _bound(P, w, s, k, e, f, C):
    """Truncation bound of the triangle plus FP64x2 rounding (a loose 2^-100)."""
    scale = np.ldexp(1.0, (e[:, None] + f[None, :]).astype(np.int64))
    trunc = k * (s + 1) * 1.01 * 2.0 ** (-s * w) * scale
    return trunc + 2.0 ** -100 * (k * scale + np.abs(C[0]))


@pytest.mark.parametrize("w,s", CONFIGS)
@pytest.mark.parametrize("variant", ["uniform", "scaled"])
def test_against_exact_rationals(w, s, variant):
    m, n, k = 4, 5, 23
    P = make_problem(m, n, k, cfg=102, variant=variant)
    hi, lo, parts = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, return_parts=True)
    exact = exact_gemm(P["A"], P["B"], P["C"])
    got = dd_value(hi, lo)
    bound = _bound(P, w, s, k, parts["e"], parts["f"], P["C"])
    worst = 0.0
    for i in range(m):
        for j in range(n):
            err = abs(got[i, j] - exact[i, j])
            assert err <= Fraction(float(bound[i, j])), (i, j, float(err), bound[i, j])
            worst = max(worst, float(err / Fraction(float(bound[i, j]))))
    if s <= 4:
        # the truncation is visible at few slices: the bound is not vacuous
        assert worst > 1e-4


def test_integer_matrices_are_exact():
    rng = np.random.default_rng(5)
    m, n, k, w = 6, 7, 40, 8
    A = rng.integers(-127, 128, (m, k)).astype(np.float64)
    B = rng.integers(-127, 128, (k, n)).astype(np.float64)
    A[:, 0] = 127.0   # row max fixes e = 7: every entry is a multiple of the first grid
    B[0, :] = -127.0
    C = rng.integers(-10 ** 6, 10 ** 6, (m, n)).astype(np.float64)
    z = np.zeros
    for s in (1, 3, 14):
        hi, lo = sl.slices_gemm((A, z((m, k))), (B, z((k, n))), (C, z((m, n))), w=w, s=s)
        assert np.array_equal(hi, A @ B + C) and np.all(lo == 0)


def test_power_of_two_row_and_column_scaling():
    P = make_problem(9, 8, 50, cfg=103)
    base = sl.slices_gemm(P["A"], P["B"], None, w=8, s=14)
    rs = np.arange(9) % 5 - 2
    cs = np.arange(8) % 3 - 1
    A2 = tuple(np.ldexp(x, rs[:, None]) for x in P["A"])
    B2 = tuple(np.ldexp(x, cs[None, :]) for x in P["B"])
    got = sl.slices_gemm(A2, B2, None, w=8, s=14)
    sh = rs[:, None] + cs[None, :]
    assert np.array_equal(got[0], np.ldexp(base[0], sh)) and np.array_equal(got[1], np.ldexp(base[1], sh))


@pytest.mark.parametrize("variant", ["uniform", "scaled"])
@pytest.mark.parametrize("w,s", [(8, 14), (9, 12)])
def test_meets_the_fp64x2_tolerance_of_the_dd_oracle(variant, w, s):
    m, n, k = 48, 40, 300
    P = make_problem(m, n, k, cfg=104, variant=variant)
    hi, lo = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s)
    rh, rl, _ = dd_gemm_ref(P["A"], P["B"], P["C"])
    AB = np.abs(P["A"][0]) @ np.abs(P["B"][0])
    err = np.abs((hi - rh) + (lo - rl))
    assert np.all(err <= 64 * k * 2.0 ** -104 * AB)
    # and per inner index as accurate as FP64x2 itself, relative to the scales
    assert np.all(err <= 2.0 ** -100 * k * np.max(np.abs(P["A"][0]), axis=1)[:, None]
                  * np.max(np.abs(P["B"][0]), axis=0)[None, :] + 2.0 ** -100 * np.abs(rh))


def test_entries_equal_full_result():
    P = make_problem(30, 20, 70, cfg=105, variant="scaled")
    hi, lo = sl.slices_gemm(P["A"], P["B"], P["C"], w=9, s=12)
    I = np.array([0, 3, 29, 17, 8])
    J = np.array([19, 0, 7, 7, 12])
    eh, el = sl.slices_gemm_entries(P["A"], P["B"], P["C"], I, J, w=9, s=12)
    assert np.array_equal(eh, hi[I, J]) and np.array_equal(el, lo[I, J])


def test_chunked_inner_dimension_stays_accurate():
    w, s = 9, 12
    k = sl.chunk_limit(w, s) + 40
    P = make_problem(2, 3, k, cfg=106)
    hi, lo = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s)
    rh, rl, _ = dd_gemm_ref(P["A"], P["B"], P["C"])
    scale = np.max(np.abs(P["A"][0]), axis=1)[:, None] * np.max(np.abs(P["B"][0]), axis=0)[None, :]
    assert np.all(np.abs((hi - rh) + (lo - rl)) <= 2.0 ** -98 * k * scale)
    eh, el = sl.slices_gemm_entries(P["A"], P["B"], P["C"], [1, 0], [2, 1], w=w, s=s)
    assert eh[0] == hi[1, 2] and el[0] == lo[1, 2] and eh[1] == hi[0, 1] and el[1] == lo[0, 1]


def test_non_finite_rows_and_columns_give_nan():
    P = make_problem(6, 5, 20, cfg=107)
    A = (P["A"][0].copy(), P["A"][1].copy())
    B = (P["B"][0].copy(), P["B"][1].copy())
    A[0][2, 3] = np.inf
    B[0][7, 4] = np.nan
    hi, lo = sl.slices_gemm(A, B, P["C"], w=8, s=14)
    assert np.all(np.isnan(hi[2, :])) and np.all(np.isnan(hi[:, 4]))
    ok = np.ones_like(hi, dtype=bool)
    ok[2, :] = False
    ok[:, 4] = False
    assert np.all(np.isfinite(hi[ok]))


def test_empty_and_zero_inner_dimension():
    P = make_problem(3, 4, 0, cfg=108)
    hi, lo = sl.slices_gemm(P["A"], P["B"], P["C"], w=8, s=14)
    assert np.array_equal(hi, P["C"][0]) and np.array_equal(lo, P["C"][1])


def test_int8_chunk_limit_keeps_level_sums_in_int32():
    for w, s in ((7, 16), (7, 15), (6, 16), (4, 9)):
        c = sl.chunk_limit(w, s, "i8")
        assert c > 0
        assert c * s * 2 ** (2 * w - 2) <= 2 ** 31 - 1
        assert c <= sl.chunk_limit(w, s)
        # maximal: one index more breaks the INT32 bound or the FP64 group bound
        assert ((c + 1) * s * 2 ** (2 * w - 2) > 2 ** 31 - 1
                or (c + 1) * s * 2 ** (2 * w - 2) * (2 ** (2 * w) + 2 ** w + 1) > 2 ** 53)
    assert sl.chunk_limit(7, 16, "i8") >= 8192


def test_int8_slices_fit_and_results_equal_the_bf16_form():
    # INT8 is the same computation as BF16 at the same (w, s) while one chunk
    # covers the inner dimension
    w, s = 7, 16
    hi, lo = _values()
    e = sl.slice_exponents(hi.reshape(1, -1), lo.reshape(1, -1), axis=1)
    slices, _ = sl.split_slices(hi.reshape(1, -1), lo.reshape(1, -1), e, 1, w, s)
    for a in slices:
        assert np.array_equal(a.astype(np.int8).astype(np.float64), a)
    P = make_problem(20, 17, 300, cfg=109, variant="scaled")
    x = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, fmt="i8")
    y = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, fmt="bf16")
    assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_int8_chunked_inner_dimension_stays_accurate():
    w, s = 5, 12
    k = sl.chunk_limit(w, s, "i8") + 100
    P = make_problem(2, 2, k, cfg=110)
    hi, lo = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, fmt="i8")
    exact_bound = k * (s + 1) * 1.01 * 2.0 ** (-s * w)
    rh, rl, _ = dd_gemm_ref(P["A"], P["B"], P["C"])
    scale = np.max(np.abs(P["A"][0]), axis=1)[:, None] * np.max(np.abs(P["B"][0]), axis=0)[None, :]
    assert np.all(np.abs((hi - rh) + (lo - rl)) <= (exact_bound + 2.0 ** -98 * k) * 2 * scale)


def _groups_model(vals):
    """sum of the weighted groups in FP64x2, every operation the rounding of
    its exact rational result, in the order the values are given."""
    h, l = 0.0, 0.0
    for v in vals:
        h, l = dd_add_d_ops(h, l, v)
    return h, l


def test_group_sum_adds_the_least_significant_group_first():
    """Groups, like the cascade's bins (Sec. 3.3, Sec. 3.6), are added from
    the least significant one up.  With w = 8 the group weights are 2^-30,
    2^-54, 2^-78, 2^-102, 2^-126; groups (2^34, 32, 0, 1, 2^24) are worth
    16, 2^-49, 0, 2^-102 and 2^-102.  From the bottom, 2^-102 + 2^-102 =
    2^-101 survives and lifts 16 + 2^-49 (a tie) upwards: the pair holds the
    exact sum 16 + 2^-49 + 2^-101.  From the top, 16 + 2^-49 rounds to 16
    with 2^-49 as the low word, which swallows each 2^-102 (ties again)."""
    w = 8
    G = [np.array([float(x)]) for x in (2 ** 34, 32, 0, 1, 2 ** 24)]
    vals = [float(g[0]) * sl.group_weight(i, w) for i, g in enumerate(G)]
    assert vals == [16.0, 2.0 ** -49, 0.0, 2.0 ** -102, 2.0 ** -102]
    h, l = sl.combine_groups(G, w)
    exact = 16 + Fraction(2) ** -49 + Fraction(2) ** -101
    assert Fraction(float(h[0])) + Fraction(float(l[0])) == exact
    assert (float(h[0]), float(l[0])) == _groups_model(vals[::-1])
    top_first = _groups_model(vals)
    assert Fraction(top_first[0]) + Fraction(top_first[1]) == 16 + Fraction(2) ** -49


def test_group_sum_matches_the_rational_model_bit_for_bit():
    """Random integer groups (magnitudes of real level-group sums, ties and
    cancellations planted) for w = 8 and w = 7: combine_groups equals the
    least-significant-first rational model; the reversed order differs on
    a good share of them."""
    rng = np.random.default_rng(78)
    for w, ng in ((8, 5), (7, 6)):
        nb = 1500
        G = [np.round(rng.uniform(-2 ** 50, 2 ** 50, nb)) for _ in range(ng)]
        q = np.arange(0, nb, 2)
        # group 1 worth exactly half an ulp of group 0 (a tie), the groups
        # below worth at most half an ulp of group 1
        v0 = G[0][q] * sl.group_weight(0, w)
        G[1][q] = np.sign(rng.uniform(-1, 1, q.size)) * 0.5 * np.spacing(np.abs(v0)) / sl.group_weight(1, w)
        for g in range(2, ng):
            lim = 0.5 * np.spacing(np.abs(G[1][q] * sl.group_weight(1, w))) / sl.group_weight(g, w)
            G[g][q] = np.round(rng.uniform(-1, 1, q.size) * np.minimum(lim, 2.0 ** 50))
        G[0][::9] = -G[0][::9]
        h, l = sl.combine_groups(G, w)
        differ = 0
        for t in range(nb):
            vals = [float(G[g][t]) * sl.group_weight(g, w) for g in range(ng)]
            want = _groups_model(vals[::-1])
            assert (float(h[t]), float(l[t])) == want, (w, t)
            differ += _groups_model(vals) != want
        assert differ > nb // 20, differ


def test_chunks_start_at_multiples_of_the_exactness_limit():
    """Chunks are added to C one by one, chunk c covering inner indices
    [c limit, (c + 1) limit).  With every chunk holding each row's and
    column's largest entry (so a chunk alone has the same powers of two as
    the whole), the result over k = 2 limit + 37 equals three slices GEMMs
    on the chunks, each adding to the previous result.  FP16, w = 11,
    s = 1: limit 2047, not a multiple of any step size; boundaries rounded
    to a multiple of 64 give different bits."""
    w, s, fmt = 11, 1, "f16"
    lim = sl.chunk_limit(w, s, fmt)
    assert lim == 2047
    k = 2 * lim + 37
    m, n = 6, 5
    rng = np.random.default_rng(112)
    A = [np.asfortranarray(rng.uniform(-0.75, 0.75, (m, k))), None]
    B = [np.asfortranarray(rng.uniform(-0.75, 0.75, (k, n))), None]
    for p0 in (0, lim, 2 * lim):
        A[0][:, p0] = 0.875
        B[0][p0, :] = -0.875
    A[1] = A[0] * 2.0 ** -53 * rng.uniform(-1, 1, (m, k))
    B[1] = B[0] * 2.0 ** -53 * rng.uniform(-1, 1, (k, n))
    C = (rng.uniform(-1, 1, (m, n)), rng.uniform(-1, 1, (m, n)) * 2.0 ** -53)
    whole = sl.slices_gemm(A, B, C, w=w, s=s, fmt=fmt)

    def by_chunks(size):
        R = C
        for p0 in range(0, k, size):
            p1 = min(k, p0 + size)
            R = sl.slices_gemm((A[0][:, p0:p1], A[1][:, p0:p1]), (B[0][p0:p1], B[1][p0:p1]), R,
                               w=w, s=s, fmt=fmt)
        return R
    got = by_chunks(lim)
    assert np.array_equal(whole[0], got[0]) and np.array_equal(whole[1], got[1])
    other = by_chunks(lim // 64 * 64)
    assert not (np.array_equal(other[0], got[0]) and np.array_equal(other[1], got[1]))
