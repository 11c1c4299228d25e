"""Pins of the numpy cascade model (CPU only).

Against: the split widths printed in Sec. 3.3; exact rounding to the digit
grid (Appendix A) computed with rationals; exact reconstruction and the
conversion bound (eq. error_scalar); exactness of bins 0-2 (Sec. 3.3-3.4)
against integer arithmetic, including worst-case digits; the worked example of
Sec. 3.6; the order of the bin sum (least significant bin first, Sec. 3.3
and Sec. 3.6) on bins where the two orders round differently; integer
matrices; the forward bound eq. (cascerr) against exact results;
row/column power-of-two invariance; identity.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cascade as cz
from oracle.ref import dd_gemm_ref
from paper_2303_04353_amd.inputs import make_problem
from tests.exact import abs_gemm, dd_add_d_ops, dd_value, exact_gemm, two_sum_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U2 = 2.0 ** -106


def test_split_widths_printed_values():
    # Sec. 3.3: k = 256 gives (22, 21, 21), 117 bits with c3 = 53; k = 64 allows c0 = 23
    assert cz.split_widths(256) == (22, 21, 21)
    assert sum(cz.split_widths(256)) + 53 == 117
    assert cz.split_widths(64)[0] == 23


@pytest.mark.parametrize("kc", [1, 2, 3, 17, 64, 100, 128, 256, 257, 512, 1024, 4096])
def test_split_widths_are_the_largest_feasible(kc):
    L = (kc - 1).bit_length()

    def ok(c0, c1, c2):
        return (2 * c0 + L <= 53 and c0 + c1 + L + 1 <= 53 and 2 * c1 + L + 2 <= 53
                and c0 + c2 + L + 2 <= 53)
    c0, c1, c2 = cz.split_widths(kc)
    assert ok(c0, c1, c2)
    assert not ok(c0 + 1, 0, 0) or not ok(c0 + 1, c1, 0)
    assert not ok(c0, c1 + 1, c2)
    assert not ok(c0, c1, c2 + 1)


def _round_to_grid(x: Fraction, g: Fraction) -> Fraction:
    return round(x / g) * g  # Fraction.__round__ rounds half to even


def _scalar_values():
    rng = np.random.default_rng(11)
    v = list(rng.uniform(-1, 1, 400))
    v += [0.0, 1.0 - 2.0 ** -53, -(1.0 - 2.0 ** -53), 0.5, -0.5, 2.0 ** -22, 2.0 ** -21,
          3 * 2.0 ** -23, 2.0 ** -60, -2.0 ** -300, 0.75 + 2.0 ** -52]
    v += list(rng.uniform(-1, 1, 100) * 2.0 ** rng.integers(-70, 0, 100))
    return np.array(v)


@pytest.mark.parametrize("kc", [64, 128, 256, 512])
def test_split_digits_are_grid_roundings(kc):
    c = cz.split_widths(kc)
    x = _scalar_values()
    d = cz.split_fp64(x, c)
    for idx in range(x.size):
        v = Fraction(float(x[idx]))
        for t in range(3):
            g = Fraction(2) ** (1 - c[t])
            want = _round_to_grid(v, g)
            assert Fraction(float(d[t][idx])) == want
            assert abs(want) <= 1
            v = (v - want) * Fraction(2) ** c[t]
        assert Fraction(float(d[3][idx])) == v  # the last digit is the exact remainder


@pytest.mark.parametrize("kc", [128, 256])
def test_split_reconstructs_fp64_exactly(kc):
    c = cz.split_widths(kc)
    s = [Fraction(1)] + [Fraction(2) ** -sum(c[:t]) for t in range(1, 4)]
    x = _scalar_values()
    d = cz.split_fp64(x, c)
    for idx in range(x.size):
        tot = sum(s[t] * Fraction(float(d[t][idx])) for t in range(4))
        assert tot == Fraction(float(x[idx]))


@pytest.mark.parametrize("kc", [128, 256])
def test_fp64x2_conversion_error_bound(kc):
    # eq. (error_scalar): the only error is the rounding of the last digit,
    # |delta| <= 2^-53 |d3| sigma_3 <= 2^-(D2+53) when |d3| <= 1
    c = cz.split_widths(kc)
    P = make_problem(6, 1, 50, cfg=80)
    hi, lo = P["A"]
    Ap, e = cz.cascade_A(hi, lo, c)
    D2 = sum(c)
    for i in range(hi.shape[0]):
        for p in range(hi.shape[1]):
            x = (Fraction(float(hi[i, p])) + Fraction(float(lo[i, p]))) * Fraction(2) ** -int(e[i])
            tot = sum(Fraction(float(Ap[t][i, p])) for t in range(4))
            d3 = abs(Fraction(float(Ap[3][i, p]))) * Fraction(2) ** D2
            err = abs(x - tot)
            assert err <= Fraction(2) ** (-53 - D2) * d3
            assert err <= Fraction(2) ** (-52 - D2)
    # matrix form (Sec. 3.4): |Sigma Delta A| <= 2 eps~ D_A J up to the same factor 2
    ell = Fraction(2) ** -(D2 + 53)
    for i in range(hi.shape[0]):
        rowmax = max(abs(Fraction(float(h))) for h in hi[i])
        for p in range(hi.shape[1]):
            val = Fraction(float(hi[i, p])) + Fraction(float(lo[i, p]))
            rec = sum(Fraction(float(Ap[t][i, p])) for t in range(4))
            err = abs(val - rec * Fraction(2) ** int(e[i]))
            assert err <= 4 * ell * rowmax


def test_exponents_bracket_the_row_max():
    P = make_problem(9, 7, 13, cfg=81, variant="scaled")
    e = cz.exponents(P["A"][0], axis=1)
    f = cz.exponents(P["B"][0], axis=0)
    for i in range(9):
        mx = np.max(np.abs(P["A"][0][i]))
        assert 2.0 ** (e[i] - 1) <= mx < 2.0 ** e[i]
    for j in range(7):
        mx = np.max(np.abs(P["B"][0][:, j]))
        assert 2.0 ** (f[j] - 1) <= mx < 2.0 ** f[j]
    z = np.zeros((3, 4))
    assert np.all(cz.exponents(z, axis=1) == 0)


@pytest.mark.parametrize("kc", [64, 128, 256, 512])
@pytest.mark.parametrize("worst", [False, True])
def test_bins_0_to_2_are_exact(kc, worst):
    # Sec. 3.3-3.4: with the widths chosen from kc, bins 0, 1 and 2 are
    # computed without error in FP64.  Checked against exact sums of the
    # digit products, with random and with worst-case (all-maximal,
    # same-sign) digits.
    c = cz.split_widths(kc)
    m = n = 3
    if worst:
        # scaled values just below 1 and with every later digit at its largest
        hi = np.full((m, kc), 1.0 - 2.0 ** -53)
        hi[:, ::2] = 0.5 + 0.5 * (1.0 - 2.0 ** -30)
        lo = hi * 2.0 ** -54
        Bh, Bl = np.asfortranarray(hi.T.copy()), np.asfortranarray(lo.T.copy())
        A = (hi, lo)
        B = (Bh, Bl)
    else:
        P = make_problem(m, n, kc, cfg=82)
        A, B = P["A"], P["B"]
    _, _, parts = cz.cascade_gemm(A, B, kc=kc, return_parts=True)
    Ap, Bp = parts["A"], parts["B"]
    bin0, bin1, bin2, _ = parts["bins"][0]
    pairs = {0: [(0, 0)], 1: [(0, 1), (1, 0)], 2: [(0, 2), (1, 1), (2, 0)]}
    for which, got in ((0, bin0), (1, bin1), (2, bin2)):
        for i in range(m):
            for j in range(n):
                s = Fraction(0)
                for (ta, tb) in pairs[which]:
                    for p in range(kc):
                        s += Fraction(float(Ap[ta][i, p])) * Fraction(float(Bp[tb][p, j]))
                assert Fraction(float(got[i, j])) == s, (which, i, j)


def _load_hex(mat):
    return np.array([[float.fromhex(v) for v in row] for row in mat])


def test_worked_example_sec3_6():
    with open(os.path.join(GOLDEN, "worked_example_sec3_6.json")) as fh:
        g = json.load(fh)
    for case in g["cases"]:
        A = (_load_hex(case["A"]["hi"]), _load_hex(case["A"]["lo"]))
        B = (_load_hex(case["B"]["hi"]), _load_hex(case["B"]["lo"]))
        hi, lo = cz.cascade_gemm(A, B, kc=256, c=case["c"])
        assert hi[0, 0] == float.fromhex(case["cascade_result"]["hi"])
        assert lo[0, 0] == float.fromhex(case["cascade_result"]["lo"])
        rh, rl, _ = dd_gemm_ref(A, B)
        assert rh[0, 0] == float.fromhex(case["fp64x2_result"]["hi"])
        assert rl[0, 0] == float.fromhex(case["fp64x2_result"]["lo"])


def test_integer_matrices_exact_over_several_blocks():
    # integers of at most 21 bits land entirely in digit 0 (grid 2^(1-c0) after
    # scaling by 2^-e with e <= 21), bins 1-6 vanish and bin 0 is exact
    rng = np.random.default_rng(5)
    m, n, k = 6, 5, 1000
    A = rng.integers(-2 ** 20, 2 ** 20 + 1, size=(m, k)).astype(float)
    B = rng.integers(-2 ** 20, 2 ** 20 + 1, size=(k, n)).astype(float)
    hi, lo = cz.cascade_gemm((A, 0 * A), (B, 0 * B), kc=256)
    want = A.astype(object) @ B.astype(object)
    assert np.all(hi.astype(object) == want) and np.all(lo == 0)


@pytest.mark.parametrize("m,n,k,variant", [(4, 3, 9, "uniform"), (5, 4, 40, "scaled"), (3, 3, 70, "uniform")])
def test_forward_bound_vs_exact(m, n, k, variant):
    # eq. (cascerr) per entry, with the rank-kc blocks accumulated in FP64x2:
    # |G - X| <= (1 + 2 nb) 2^-106 (|A||B|)_ij + 40 kc k eps~ ||a_i|| ||b_j|| (+ C rounding)
    kc = 16
    P = make_problem(m, n, k, cfg=83, variant=variant)
    hi, lo = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc)
    X = exact_gemm(P["A"], P["B"], P["C"])
    S = abs_gemm(P["A"], P["B"])
    Cabs = np.abs(dd_value(*P["C"]))
    c = cz.split_widths(kc)
    eps_t = Fraction(2) ** -(sum(c) + 53)
    nb = -(-k // kc)
    a = dd_value(*P["A"])
    b = dd_value(*P["B"])
    G = dd_value(hi, lo)
    for i in range(m):
        ai = max(abs(v) for v in a[i])
        for j in range(n):
            bj = max(abs(v) for v in b[:, j])
            bound = ((1 + 2 * nb) * Fraction(U2) * S[i, j] + 40 * kc * k * eps_t * ai * bj
                     + 4 * Fraction(U2) * (Cabs[i, j] + S[i, j]))
            assert abs(G[i, j] - X[i, j]) <= bound


def test_row_and_column_power_of_two_invariance_bitwise():
    P = make_problem(12, 9, 300, cfg=84)
    A, B, C = P["A"], P["B"], P["C"]
    r = np.arange(12) % 7 - 3
    s = np.arange(9) % 5 - 2
    h0, l0 = cz.cascade_gemm(A, B, C, kc=128)
    Ar = (np.ldexp(A[0], r[:, None]), np.ldexp(A[1], r[:, None]))
    Bs = (np.ldexp(B[0], s[None, :]), np.ldexp(B[1], s[None, :]))
    sh = r[:, None] + s[None, :]
    Cs = (np.ldexp(C[0], sh), np.ldexp(C[1], sh))
    h1, l1 = cz.cascade_gemm(Ar, Bs, Cs, kc=128)
    assert np.array_equal(h1, np.ldexp(h0, sh)) and np.array_equal(l1, np.ldexp(l0, sh))


def test_identity_within_conversion_error():
    k, n = 8, 6
    P = make_problem(k, n, k, cfg=85)
    B = P["B"]
    hi, lo = cz.cascade_gemm((np.eye(k), np.zeros((k, k))), B, kc=256)
    c = cz.split_widths(k)
    ell = Fraction(2) ** -(sum(c) + 53)
    got = dd_value(hi, lo)
    want = dd_value(*B)
    for j in range(n):
        bj = max(abs(v) for v in want[:, j])
        for i in range(k):
            assert abs(got[i, j] - want[i, j]) <= 8 * ell * bj


def test_agrees_with_fp64x2_oracle_within_tolerance():
    m = n = k = 128
    P = make_problem(m, n, k, cfg=0)
    hi, lo = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=256)
    rh, rl, _ = dd_gemm_ref(P["A"], P["B"], P["C"])
    diff = (hi - rh) + (lo - rl)
    AB = np.abs(P["A"][0]) @ np.abs(P["B"][0])
    assert np.all(np.abs(diff) <= 64 * k * 2.0 ** -104 * AB)


def test_derived_B_planes_are_single_roundings():
    # B4' = sigma_2 B4 = B2' + B3', B5' = sigma_1 B5 = B1' + B2' + B3' (through
    # B4'), B6 = the scaled FP64x2 entry itself (Sec. 3.4); each is the exact
    # sum rounded once to FP64 (Python's float(Fraction) rounds correctly).
    P = make_problem(5, 40, 33, cfg=86)
    hi, lo = P["B"]
    c = cz.split_widths(256)
    Bp, f = cz.cascade_B(hi, lo, c)
    nb6 = 0
    for p in range(hi.shape[0]):
        for j in range(hi.shape[1]):
            q = [Fraction(float(Bp[t][p, j])) for t in range(7)]
            assert q[4] == Fraction(float(q[2] + q[3]))
            assert q[5] == Fraction(float(q[1] + q[4]))
            y = (Fraction(float(hi[p, j])) + Fraction(float(lo[p, j]))) * Fraction(2) ** -int(f[j])
            assert q[6] == Fraction(float(y))
            nb6 += q[6] != Fraction(float(hi[p, j])) * Fraction(2) ** -int(f[j])
    assert nb6 > 0  # the low word changes B6' for some entries


def test_cancellation_flag_on_the_worked_example():
    # Sec. 3.6: x = (1, eps), y = (0, 1): the leading digits' product is zero
    # while the last bin carries eps, and the cascade loses eps's low word
    # (Sec. 3.7: zeros in bin 0 flag results subject to cancellation error).
    case = json.load(open(os.path.join(GOLDEN, "worked_example_sec3_6.json")))["cases"][0]
    h = lambda v: np.array([[float.fromhex(x) for x in row] for row in v])
    A = (h(case["A"]["hi"]), h(case["A"]["lo"]))
    B = (h(case["B"]["hi"]), h(case["B"]["lo"]))
    hi, lo, parts = cz.cascade_gemm(A, B, c=tuple(case["c"]), return_parts=True)
    assert cz.cancellation_flags(parts["bins"])[0, 0]
    assert hi[0, 0] == float.fromhex(case["cascade_result"]["hi"])


def test_cancellation_flags_constructed_and_random():
    rng = np.random.default_rng(4)
    m, n, k = 6, 5, 40
    Ahi = rng.uniform(-1, 1, (m, k))
    Bhi = rng.uniform(-1, 1, (k, n))
    z = np.zeros
    # row 2 of A and column 3 of B agree in their leading digits up to a sign
    # flip in half the terms: the leading products cancel exactly, the rest not
    Ahi[2, :] = 0.75
    Ahi[2, 1::2] = 0.75 + 2.0 ** -30
    Bhi[:, 3] = 0.5
    Bhi[1::2, 3] = -0.5
    # row 4 of A is zero: its products are exactly zero, no risk
    Ahi[4, :] = 0.0
    hi, lo, parts = cz.cascade_gemm((Ahi, z((m, k))), (Bhi, z((k, n))), kc=16, return_parts=True)
    flags = cz.cancellation_flags(parts["bins"])
    assert flags[2, 3]
    # the result itself is the small difference: 20 * 2^-30 * 0.5 with the sign of the odd terms
    assert hi[2, 3] == -20 * 2.0 ** -31
    assert not flags[4].any()
    others = np.ones_like(flags)
    others[2, 3] = False
    assert not flags[others].any()


# --- Sigma and T per rank-kc panel (scaling="panel") ------------------------------

def test_panel_scaling_equals_global_for_one_block():
    P = make_problem(9, 7, 50, cfg=86, variant="scaled")
    for kc in (50, 64, 256):
        a = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc)
        b = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc, scaling="panel")
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_panel_scaling_equals_global_when_panel_maxima_share_the_exponent():
    # every panel of every row (column) holds an entry in the row's (column's)
    # top binade, so the panel exponents equal the global ones: scaling each
    # block exactly by the same powers of two before or after the FP64x2
    # accumulation gives the same bits
    m, n, k, kc = 10, 8, 100, 16
    P = make_problem(m, n, k, cfg=87, variant="scaled")
    A, B = [x.copy() for x in P["A"]], [x.copy() for x in P["B"]]
    for p0 in range(0, k, kc):
        A[0][:, p0] = 0.99 * np.ldexp(1.0, cz.exponents(P["A"][0], axis=1)) * 0.75
        B[0][p0, :] = -0.99 * np.ldexp(1.0, cz.exponents(P["B"][0], axis=0)) * 0.75
    A[1][:, ::kc] = 0.0
    B[1][::kc, :] = 0.0
    _, _, parts = cz.cascade_gemm(A, B, P["C"], kc=kc, scaling="panel", return_parts=True)
    eg, fg = cz.exponents(A[0], axis=1), cz.exponents(B[0], axis=0)
    assert np.all(parts["e"] == eg[None, :]) and np.all(parts["f"] == fg[None, :])
    a = cz.cascade_gemm(A, B, P["C"], kc=kc)
    b = cz.cascade_gemm(A, B, P["C"], kc=kc, scaling="panel")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_panel_scaling_is_invariant_to_power_of_two_balancing():
    # A F F^-1 B with F a power of two constant over each panel (Sec. 6,
    # scaling/balancing): per-panel exponents absorb F exactly, bit for bit
    m, n, k, kc = 11, 9, 90, 32
    P = make_problem(m, n, k, cfg=88)
    pan = np.arange(k) // kc
    t = np.array([7, -12, 30])[pan]
    Af = (np.ldexp(P["A"][0], t[None, :]), np.ldexp(P["A"][1], t[None, :]))
    Bf = (np.ldexp(P["B"][0], -t[:, None]), np.ldexp(P["B"][1], -t[:, None]))
    a = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc, scaling="panel")
    b = cz.cascade_gemm(Af, Bf, P["C"], kc=kc, scaling="panel")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # with one exponent per row the balancing changes the result
    g = cz.cascade_gemm(Af, Bf, P["C"], kc=kc)
    h = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc)
    assert not (np.array_equal(g[0], h[0]) and np.array_equal(g[1], h[1]))


@pytest.mark.parametrize("m,n,k,kc", [(4, 3, 24, 8), (5, 4, 40, 16), (3, 5, 33, 8)])
def test_panel_scaling_forward_bound_vs_exact(m, n, k, kc):
    # eq. (cascerr) per panel: each block's bound uses that panel's row and
    # column maxima, so on data whose scale changes along k the sum of panel
    # bounds stays near (|A||B|)_ij, where one exponent per row does not
    P = make_problem(m, n, k, cfg=89, variant="panels", panel=kc)
    hi, lo = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc, scaling="panel")
    X = exact_gemm(P["A"], P["B"], P["C"])
    S = abs_gemm(P["A"], P["B"])
    Cabs = np.abs(dd_value(*P["C"]))
    c = cz.split_widths(kc)
    eps_t = Fraction(2) ** -(sum(c) + 53)
    nb = -(-k // kc)
    a = dd_value(*P["A"])
    b = dd_value(*P["B"])
    G = dd_value(hi, lo)
    for i in range(m):
        for j in range(n):
            panel_term = Fraction(0)
            for p0 in range(0, k, kc):
                ai = max(abs(v) for v in a[i, p0:p0 + kc])
                bj = max(abs(v) for v in b[p0:p0 + kc, j])
                panel_term += 40 * kc * kc * eps_t * ai * bj
            bound = ((1 + 2 * nb) * Fraction(U2) * S[i, j] + panel_term
                     + 4 * Fraction(U2) * (Cabs[i, j] + S[i, j]))
            assert abs(G[i, j] - X[i, j]) <= bound


def test_panel_scaling_meets_the_tolerance_where_global_scaling_does_not():
    # rows large in the first panel and small in the second, columns the other
    # way round: every product is small, and one exponent per row or column
    # leaves the small halves with FP64 digits only
    m = n = 6
    kc, k = 16, 32
    rng = np.random.default_rng(9)
    Ahi = rng.uniform(-1, 1, (m, k))
    Bhi = rng.uniform(-1, 1, (k, n))
    Ahi[:, kc:] *= 2.0 ** -90
    Bhi[:kc, :] *= 2.0 ** -90
    A = (Ahi, Ahi * 2.0 ** -53 * rng.uniform(-1, 1, (m, k)))
    B = (Bhi, Bhi * 2.0 ** -53 * rng.uniform(-1, 1, (k, n)))
    X = exact_gemm(A, B)
    tol = 64 * k * Fraction(2) ** -104 * abs_gemm(A, B)
    Gp = dd_value(*cz.cascade_gemm(A, B, kc=kc, scaling="panel"))
    Gg = dd_value(*cz.cascade_gemm(A, B, kc=kc))
    assert all(abs(Gp[idx] - X[idx]) <= tol[idx] for idx in np.ndindex(m, n))
    assert sum(abs(Gg[idx] - X[idx]) > tol[idx] for idx in np.ndindex(m, n)) > m * n // 2


def test_panel_scaling_ragged_last_panel_and_zero_panels():
    m, n, k, kc = 7, 5, 45, 16
    P = make_problem(m, n, k, cfg=90, variant="panels", panel=kc)
    A = [x.copy() for x in P["A"]]
    A[0][2, 16:32] = 0.0
    A[1][2, 16:32] = 0.0
    hi, lo, parts = cz.cascade_gemm(A, P["B"], P["C"], kc=kc, scaling="panel", return_parts=True)
    assert parts["e"].shape == (3, m) and parts["f"].shape == (3, n)
    assert parts["e"][1, 2] == 0
    rh, rl, _ = dd_gemm_ref(A, P["B"], P["C"])
    AB = np.abs(A[0]) @ np.abs(P["B"][0])
    assert np.all(np.abs((hi - rh) + (lo - rl)) <= 64 * k * 2.0 ** -104 * AB)


# --- power-of-two diagonal balancing F (balance=True) ------------------------------

def test_balancing_is_the_identity_on_balanced_operands():
    # column maxima of A and row maxima of B in the same binade: F = I
    P = make_problem(12, 9, 70, cfg=91)
    A = [x.copy() for x in P["A"]]
    B = [x.copy() for x in P["B"]]
    A[0][0, :], A[1][0, :] = 0.75, 0.0
    B[0][:, 0], B[1][:, 0] = -0.75, 0.0
    assert np.all(cz.balance_exponents(A[0], B[0]) == 0)
    a = cz.cascade_gemm(A, B, P["C"], kc=32)
    b = cz.cascade_gemm(A, B, P["C"], kc=32, balance=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_balancing_evens_out_columns_of_A_and_rows_of_B():
    P = make_problem(20, 15, 60, cfg=92, variant="skewed")
    g = cz.balance_exponents(P["A"][0], P["B"][0])
    A2 = np.ldexp(P["A"][0], g[None, :])
    B2 = np.ldexp(P["B"][0], -g[:, None])
    eA = cz.exponents(A2, axis=0)
    eB = cz.exponents(B2, axis=1)
    assert np.all(np.abs(eA - eB) <= 1)
    # the skew of the inputs is large before
    assert np.max(np.abs(cz.exponents(P["A"][0], axis=0) - cz.exponents(P["B"][0], axis=1))) > 40


def test_balancing_exponents_absorb_any_power_of_two_diagonal():
    # g(A F0, F0^-1 B) = g(A, B) - f0 for every integer f0_p: the balanced
    # operands do not depend on F0 (a rounding of (e_B - e_A)/2 toward zero
    # would break this for odd differences)
    P = make_problem(9, 7, 400, cfg=96, variant="skewed")
    A, B = P["A"][0], P["B"][0]
    g = cz.balance_exponents(A, B)
    rng = np.random.default_rng(4)
    for _ in range(5):
        f0 = rng.integers(-50, 51, size=400)
        g2 = cz.balance_exponents(np.ldexp(A, f0[None, :]), np.ldexp(B, -f0[:, None]))
        assert np.array_equal(g2, g - f0)


@pytest.mark.parametrize("scaling", ["global", "panel"])
def test_balanced_cascade_is_invariant_to_power_of_two_diagonal_scaling(scaling):
    # (A F0, F0^-1 B) balances to the same operands as (A, B), bit for bit
    m, n, k, kc = 10, 8, 90, 32
    P = make_problem(m, n, k, cfg=93, variant="skewed")
    f0 = (np.arange(k) * 37 % 61) - 30
    Af = tuple(np.ldexp(x, f0[None, :]) for x in P["A"])
    Bf = tuple(np.ldexp(x, -f0[:, None]) for x in P["B"])
    a = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc, scaling=scaling, balance=True)
    b = cz.cascade_gemm(Af, Bf, P["C"], kc=kc, scaling=scaling, balance=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    u = cz.cascade_gemm(P["A"], P["B"], P["C"], kc=kc, scaling=scaling)
    v = cz.cascade_gemm(Af, Bf, P["C"], kc=kc, scaling=scaling)
    assert not (np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1]))


def test_balancing_meets_the_tolerance_on_skewed_operands():
    # rows of A and columns of B take their scale from the most skewed inner
    # index, so without balancing most products have FP64 digits only
    m, n, k = 6, 5, 40
    P = make_problem(m, n, k, cfg=94, variant="skewed")
    X = exact_gemm(P["A"], P["B"], P["C"])
    S = abs_gemm(P["A"], P["B"]) + np.abs(dd_value(*P["C"]))
    tol = 64 * k * Fraction(2) ** -104 * S
    Gb = dd_value(*cz.cascade_gemm(P["A"], P["B"], P["C"], kc=16, balance=True))
    Gu = dd_value(*cz.cascade_gemm(P["A"], P["B"], P["C"], kc=16))
    assert all(abs(Gb[idx] - X[idx]) <= tol[idx] for idx in np.ndindex(m, n))
    assert sum(abs(Gu[idx] - X[idx]) > tol[idx] for idx in np.ndindex(m, n)) > m * n // 2


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_balancing_with_zero_and_non_finite_slices():
    m, n, k = 7, 6, 30
    P = make_problem(m, n, k, cfg=95, variant="skewed")
    A = [x.copy() for x in P["A"]]
    A[0][:, 3] = 0.0
    A[1][:, 3] = 0.0
    hi, lo = cz.cascade_gemm(A, P["B"], P["C"], kc=16, balance=True)
    rh, rl, _ = dd_gemm_ref(A, P["B"], P["C"])
    AB = np.abs(A[0]) @ np.abs(P["B"][0]) + np.abs(P["C"][0])
    assert np.all(np.abs((hi - rh) + (lo - rl)) <= 64 * k * 2.0 ** -104 * AB)
    A[0][2, 5] = np.inf
    hi, lo = cz.cascade_gemm(A, P["B"], P["C"], kc=16, balance=True)
    assert np.all(np.isnan(hi[2, :])) and np.all(np.isfinite(np.delete(hi, 2, axis=0)))


def _bins_lsf_model(b0, b1, b2, b36):
    """bin0 + (bin1 + (bin2 + bin36)) with every operation taken as the
    rounding of its exact rational result (Sec. 3.6's expression for
    fl_casc; the bins are summed least significant first)."""
    h, l = two_sum_exact(b2, b36)
    h, l = dd_add_d_ops(h, l, b1)
    return dd_add_d_ops(h, l, b0)


def _bins_msf_model(b0, b1, b2, b36):
    """The reversed order, bin 0 first: what a wrong order would give."""
    h, l = two_sum_exact(b0, b1)
    h, l = dd_add_d_ops(h, l, b2)
    return dd_add_d_ops(h, l, b36)


def test_bin_sum_adds_the_least_significant_bin_first():
    """Sec. 3.3 and Sec. 3.6 add the bins from the least significant one up.
    Bins 1, 2^-53, 2^-106, 2^-106: adding bin 0 first rounds 1 + 2^-53 to
    the even 1 and keeps 2^-53 as the low word, which then swallows each
    2^-106 (a tie again).  Added from the bottom, 2^-106 + 2^-106 = 2^-105
    survives, lifts 1 + 2^-53 above the tie, and the pair holds the exact
    sum 1 + 2^-53 + 2^-105."""
    arr = lambda *v: [np.array([x]) for x in v]
    b = (1.0, 2.0 ** -53, 2.0 ** -106, 2.0 ** -106)
    h, l = cz.combine_bins(*arr(*b))
    exact = Fraction(1) + Fraction(2) ** -53 + Fraction(2) ** -105
    assert Fraction(float(h[0])) + Fraction(float(l[0])) == exact
    assert (float(h[0]), float(l[0])) == (1.0 + 2.0 ** -52, -2.0 ** -53 + 2.0 ** -105)
    rh, rl = _bins_msf_model(*b)
    assert Fraction(rh) + Fraction(rl) == 1 + Fraction(2) ** -53      # the other order loses 2^-105
    # with total cancellation of the leading bins the least-significant-first
    # order loses the smallest bin instead: bins 1, -1, 2^-60, 2^-120 give
    # 2^-60 exactly (bin2 + bin36 = 2^-60 + 2^-120 is kept as a pair, adding
    # -1 moves 2^-60 to the low word, where 2^-120 rounds away)
    h, l = cz.combine_bins(*arr(1.0, -1.0, 2.0 ** -60, 2.0 ** -120))
    assert (float(h[0]), float(l[0])) == (2.0 ** -60, 0.0)
    assert _bins_msf_model(1.0, -1.0, 2.0 ** -60, 2.0 ** -120) == (2.0 ** -60, 2.0 ** -120)
    # bin 2 before bin 1: bins 1, -1, 2^-54, 3 2^-107.  bin2 + bin36 rounds
    # (a tie) to 2^-54 + 2^-105 and keeps -2^-107; adding -1 and 1 then
    # leaves the pair exact: 2^-54 + 3 2^-107.  Taking bin 1 with bin 3-6
    # first loses the -2^-107 when 1 and -1 meet.
    b = (1.0, -1.0, 2.0 ** -54, 3 * 2.0 ** -107)
    h, l = cz.combine_bins(*arr(*b))
    exact = Fraction(2) ** -54 + 3 * Fraction(2) ** -107
    assert Fraction(float(h[0])) + Fraction(float(l[0])) == exact
    hs, ls = two_sum_exact(b[1], b[3])
    hs, ls = dd_add_d_ops(hs, ls, b[2])
    hs, ls = dd_add_d_ops(hs, ls, b[0])
    assert Fraction(hs) + Fraction(ls) != exact


def test_fp64x2_addition_keeps_both_low_words():
    """The accurate FP64x2 addition (used for the rank-kc accumulation and
    for C) adds the low words with an error-free sum and folds its error in
    last.  When the high words cancel, that error is the result's low word:
    (1, 2^-60) + (-1, 3 2^-114) = 2^-60 + 3 2^-114 exactly, held as
    (2^-60 + 2^-112, -2^-114).  On random pairs with heavy cancellation the
    relative error stays within 3 2^-106, the published bound of this
    algorithm (Joldes, Muller and Popescu, 2017: AccurateDWPlusDW)."""
    h, l = cz.dd_add(np.array([1.0]), np.array([2.0 ** -60]), np.array([-1.0]), np.array([3 * 2.0 ** -114]))
    assert (float(h[0]), float(l[0])) == (2.0 ** -60 + 2.0 ** -112, -2.0 ** -114)
    rng = np.random.default_rng(79)
    n = 20000
    xh = rng.uniform(-1, 1, n) * np.ldexp(1.0, rng.integers(-20, 20, n))
    xl = xh * rng.uniform(-1, 1, n) * 2.0 ** -53
    xh, xl = cz.quick_two_sum(xh, xl)              # canonical pairs
    # y close to -x: high words cancel to a few bits
    yh = -xh * (1 + rng.integers(-8, 9, n) * 2.0 ** -52)
    yl = yh * rng.uniform(-1, 1, n) * 2.0 ** -53
    yh, yl = cz.quick_two_sum(yh, yl)
    h, l = cz.dd_add(xh, xl, yh, yl)
    for t in range(n):
        exact = Fraction(float(xh[t])) + Fraction(float(xl[t])) + Fraction(float(yh[t])) + Fraction(float(yl[t]))
        err = abs(Fraction(float(h[t])) + Fraction(float(l[t])) - exact)
        assert err <= 3 * Fraction(2) ** -106 * abs(exact), t


def test_bin_sum_matches_the_rational_model_bit_for_bit():
    """Random bins with the magnitudes of a rank-kc block (bin L near
    2^-21 L, bin 3-6 near 2^-64, on the grids of the split), plus planted
    cancellation and ties: combine_bins equals the operation-by-operation
    rational model of the least-significant-first order, and on the cases
    where the reversed order differs it is the first that is returned."""
    rng = np.random.default_rng(77)
    nb = 4000
    b0 = np.ldexp(np.round(rng.uniform(-2 ** 44, 2 ** 44, nb)), -44)
    b1 = np.ldexp(np.round(rng.uniform(-2 ** 52, 2 ** 52, nb)), -74)
    b2 = np.ldexp(np.round(rng.uniform(-2 ** 52, 2 ** 52, nb)), -96)
    b36 = np.ldexp(rng.uniform(-1, 1, nb), -64)
    b0[::7] = -np.round(b1[::7] * 2 ** 22) * 2.0 ** -22           # bin 0 cancels bin 1's top
    b1[::5] = 0.0
    b36[::11] = np.ldexp(np.sign(b0[::11]) * 0.5, -52) * np.abs(b0[::11])   # ties with bin 0's ulp
    # every third entry: bin 1 exactly half an ulp of bin 0 (a tie), bins 2
    # and 3-6 each at most half an ulp of bin 1, of random signs
    q = np.arange(0, nb, 3)
    u0 = np.spacing(np.abs(b0[q]))
    b1[q] = np.where(rng.uniform(size=q.size) < 0.5, -0.5, 0.5) * u0
    u1 = np.spacing(np.abs(b1[q]))
    b2[q] = np.where(rng.uniform(size=q.size) < 0.5, -0.5, 0.5) * u1 * rng.integers(0, 2, q.size)
    b36[q] = np.where(rng.uniform(size=q.size) < 0.5, -0.5, 0.5) * u1 * rng.choice([0.5, 1.0, 0.75], q.size)
    h, l = cz.combine_bins(b0, b1, b2, b36)
    differ = 0
    for t in range(nb):
        want = _bins_lsf_model(float(b0[t]), float(b1[t]), float(b2[t]), float(b36[t]))
        assert (float(h[t]), float(l[t])) == want, t
        differ += _bins_msf_model(float(b0[t]), float(b1[t]), float(b2[t]), float(b36[t])) != want
    assert differ > nb // 20   # the test can tell the two orders apart
