"""Pins of the FP64x3 cascade model (CPU only).

Against: the exactness rule behind the split widths and their maximality;
exact reconstruction of every entry from its six digits (rationals); bins
0..4 equal to exact sums, including worst-case digits; the suffix planes as
rounded running sums; the triple-word rounding against hand-worked values
and against rationals, with cancellation (also across several levels);
results against exact rational
C + A B within the analogue of eq. (cascerr); integer matrices; power-of-two
row/column invariance; k = 0.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import cascade3 as c3
from paper_2303_04353_amd.inputs import make_problem3

F = Fraction
U3 = F(1, 2 ** 159)


def _val(ws, idx):
    return sum(F(float(w[idx])) for w in ws)


@pytest.mark.parametrize("kc", [4, 64, 256, 1024])
def test_widths_satisfy_the_rule_and_are_locally_maximal(kc):
    c = c3.widths3(kc)
    assert c3.exact_bins_ok(c, kc)
    for t in range(5):
        wider = list(c)
        wider[t] += 1
        assert not c3.exact_bins_ok(tuple(wider), kc), (kc, t)
    # wider blocks need narrower digits
    if kc > 4:
        assert sum(c) <= sum(c3.widths3(kc // 4))


def test_split_reconstructs_every_entry():
    kc = 64
    c = c3.widths3(kc)
    P = make_problem3(7, 9, 5, cfg=1)
    e = c3.exponents(P["A"][0], axis=1)
    planes, scaled = c3.split3(P["A"], e, 1, c)
    for idx in np.ndindex(7, 5):
        v = _val(scaled, idx)
        got = sum(F(float(p[idx])) for p in planes)
        # levels 0..4 exact; the remainder level rounds twice (two additions)
        assert abs(got - v) <= 2 * F(2) ** -(sum(c) + 53) * 4, idx
        # every digit on its grid and within 3 of its level
        Dc = np.cumsum(c)
        for t in range(5):
            d = F(float(planes[t][idx])) * F(2) ** (int(Dc[t - 1]) if t else 0)
            step = F(2) ** (1 - c[t])
            assert (d / step).denominator == 1 and abs(d) <= 3, (idx, t)


def test_bins_0_to_4_are_exact_with_worst_case_digits():
    kc = 256
    c = c3.widths3(kc)
    Dc = np.cumsum(c)
    Dm = [0] + list(Dc[:-1])
    rng = np.random.default_rng(2)
    m = n = 3
    # digits at the largest magnitude the split can produce: 3 in units of
    # the level, on the level's grid, random signs
    def planes(shape):
        out = []
        for t in range(5):
            steps = 3 * 2 ** (c[t] - 1)
            ints = rng.integers(steps - 2, steps + 1, size=shape) * np.where(rng.uniform(size=shape) < 0.5, -1, 1)
            out.append(np.ldexp(ints.astype(float), int(1 - c[t] - Dm[t])))
        out.append(np.ldexp(rng.uniform(-3, 3, size=shape), -int(Dc[4])))
        return out
    for same_sign in (False, True):
        Ap, Bp = planes((m, kc)), planes((kc, n))
        if same_sign:
            Ap = [np.abs(x) for x in Ap]
            Bp = [np.abs(x) for x in Bp]
        U = c3.suffix_planes(Bp)
        bins = c3.bins3_block(Ap, Bp, U, 0, kc)
        for L in range(5):
            for i in range(m):
                for j in range(n):
                    want = sum(F(float(Ap[a][i, p])) * F(float(Bp[L - a][p, j]))
                               for a in range(L + 1) for p in range(kc))
                    assert F(float(bins[L][i, j])) == want, (L, i, j, same_sign)


def _ulp(x):
    return F(float(np.spacing(abs(x)))) if x != 0 else F(0)


def _check_round3(vals, words):
    """The words are the rounding of the exact sum S: w0 within half an ulp
    of S, w1 within half an ulp of S - w0, w2 within half an ulp of
    S - w0 - w1 (each the nearest double to what is left)."""
    S = sum(F(v) for v in vals)
    w0, w1, w2 = (float(x) for x in words)
    for w, rest in ((w0, S), (w1, S - F(w0)), (w2, S - F(w0) - F(w1))):
        assert abs(F(w) - rest) <= _ulp(w) / 2 or (w == 0.0 and rest == 0), (vals, words)
    return S


def test_triple_word_rounding_closed_forms():
    """Values whose triple-word rounding is known by hand: non-overlapping
    powers of two keep their first three, a tie goes to the even neighbour,
    a complete cancellation leaves the small terms."""
    one = lambda *v: c3.td_round([np.array([x]) for x in v])
    got = one(1.0, 2.0 ** -60, 2.0 ** -120, 2.0 ** -180)
    assert tuple(float(x[0]) for x in got) == (1.0, 2.0 ** -60, 2.0 ** -120)
    got = one(2.0 ** -180, 2.0 ** -120, 2.0 ** -60, 1.0)          # order does not matter
    assert tuple(float(x[0]) for x in got) == (1.0, 2.0 ** -60, 2.0 ** -120)
    got = one(1.0, -1.0, 2.0 ** -70, 2.0 ** -140, 2.0 ** -200)
    assert tuple(float(x[0]) for x in got) == (2.0 ** -70, 2.0 ** -140, 2.0 ** -200)
    # 1 + 2^-53 is a tie between 1 and 1 + 2^-52: the even one, 1, with 2^-53 left
    got = one(1.0, 2.0 ** -53)
    assert tuple(float(x[0]) for x in got) == (1.0, 2.0 ** -53, 0.0)
    # 1 + 2^-53 + 2^-110 is above the tie: rounds up, the rest is negative
    got = one(1.0, 2.0 ** -53, 2.0 ** -110)
    assert tuple(float(x[0]) for x in got) == (1.0 + 2.0 ** -52, -2.0 ** -53, 2.0 ** -110)
    got = one(0.0, 0.0)
    assert tuple(float(x[0]) for x in got) == (0.0, 0.0, 0.0)
    got = one(1.0, np.nan)
    assert all(np.isnan(x[0]) for x in got)


def test_triple_word_sum_against_rationals():
    rng = np.random.default_rng(3)
    for trial in range(300):
        n = int(rng.integers(2, 10))
        ex = rng.integers(-120, 20, size=n)
        terms = [np.array([float(np.ldexp(rng.uniform(-1, 1), int(e)))]) for e in ex]
        if trial % 3 == 0:   # planted cancellation: a term and its negation
            terms.append(-terms[0] * (1 + 2.0 ** -40))
        r = c3.td_round(terms)
        vals = [float(t[0]) for t in terms]
        S = _check_round3(vals, [x[0] for x in r])
        got = sum(F(float(x[0])) for x in r)
        assert abs(got - S) <= F(1, 2 ** 158) * abs(S), trial
        # the words do not overlap
        r0, r1, r2 = (float(x[0]) for x in r)
        assert abs(r1) <= abs(np.spacing(r0)) / 2 and abs(r2) <= abs(np.spacing(r1)) / 2 + 1e-320


def test_triple_word_sum_with_multilevel_cancellation():
    """A triple word plus pairs of large terms that cancel up to a small
    remainder (up to 2^60 above the sum), in random order: the three words
    hold the exact sum to 2^-158 relative, whatever the order."""
    rng = np.random.default_rng(8)
    for trial in range(500):
        n = int(rng.integers(3, 13))
        s0 = rng.uniform(-1, 1)
        vals = [s0, s0 * 2.0 ** -60 * rng.uniform(-1, 1), s0 * 2.0 ** -120 * rng.uniform(-1, 1)]
        while len(vals) < n:
            big = float(np.ldexp(rng.uniform(0.5, 1), int(rng.integers(1, 60)))) * float(rng.choice([-1, 1]))
            small = float(np.ldexp(rng.uniform(-1, 1), int(rng.integers(-170, -1))))
            vals += [big, -big + small]
        vals = [vals[i] for i in rng.permutation(n)]
        got = c3.td_round([np.array([v]) for v in vals])
        S = _check_round3(vals, [x[0] for x in got])
        assert abs(sum(F(float(x[0])) for x in got) - S) <= F(1, 2 ** 158) * abs(S), trial
        rev = c3.td_round([np.array([v]) for v in vals[::-1]])
        assert all(float(a[0]) == float(b[0]) for a, b in zip(got, rev))


def test_suffix_planes_are_rounded_running_sums():
    """U_5' = B_5', and each U_t' is within (5 - t) roundings of the exact
    sum B_t' + ... + B_5' (one rounding per addition); U_0' is the scaled
    entry to within a few of its ulps, since the planes rebuild it."""
    kc = 64
    c = c3.widths3(kc)
    P = make_problem3(3, 9, kc, cfg=11, variant="scaled")
    f = c3.exponents(P["B"][0], axis=0)
    Bp, scaled = c3.split3(P["B"], f, 0, c)
    U = c3.suffix_planes(Bp)
    assert np.array_equal(U[5], Bp[5])
    for idx in np.ndindex(kc, 9):
        for t in range(5):
            exact = sum(F(float(Bp[s][idx])) for s in range(t, 6))
            err = abs(F(float(U[t][idx])) - exact)
            assert err <= (5 - t) * _ulp(float(U[t][idx])), (idx, t)
            # every plane contributes: dropping the last one shows
            if Bp[5][idx] != 0 and t == 4:
                assert F(float(U[4][idx])) != F(float(Bp[4][idx])) or abs(Bp[5][idx]) < np.spacing(abs(Bp[4][idx]))
        v = _val(scaled, idx)
        assert abs(F(float(U[0][idx])) - v) <= 3 * _ulp(float(U[0][idx])), idx


@pytest.mark.parametrize("m,n,k,kc,variant", [(5, 4, 40, 16, "uniform"), (4, 6, 70, 32, "scaled"),
                                              (3, 3, 9, 256, "uniform")])
def test_results_within_the_forward_bound(m, n, k, kc, variant):
    P = make_problem3(m, n, k, cfg=4, variant=variant)
    R = c3.cascade3_gemm(P["A"], P["B"], P["C"], kc=kc)
    kce = min(kc, k)
    eps = F(c3.eps3(kce))
    nb = -(-k // kce)
    for i in range(m):
        for j in range(n):
            a = [_val(P["A"], (i, p)) for p in range(k)]
            b = [_val(P["B"], (p, j)) for p in range(k)]
            X = sum(x * y for x, y in zip(a, b)) + _val(P["C"], (i, j))
            S = sum(abs(x * y) for x, y in zip(a, b))
            Cabs = abs(_val(P["C"], (i, j)))
            bound = ((1 + 4 * nb) * 8 * U3 * S + 40 * kce * k * eps * max(map(abs, a)) * max(map(abs, b))
                     + 8 * U3 * (Cabs + S))
            assert abs(_val(R, (i, j)) - X) <= bound, (i, j)


def test_integer_matrices_exact():
    rng = np.random.default_rng(5)
    m, n, k = 5, 4, 300
    A = rng.integers(-2 ** 20, 2 ** 20 + 1, size=(m, k)).astype(float)
    B = rng.integers(-2 ** 20, 2 ** 20 + 1, size=(k, n)).astype(float)
    z = lambda s: np.zeros(s)
    R = c3.cascade3_gemm((A, z(A.shape), z(A.shape)), (B, z(B.shape), z(B.shape)), kc=64)
    want = A.astype(object) @ B.astype(object)
    assert np.all(R[0].astype(object) == want) and np.all(R[1] == 0) and np.all(R[2] == 0)


def test_power_of_two_row_and_column_invariance():
    P = make_problem3(6, 5, 90, cfg=6)
    r = np.arange(6) % 5 - 2
    s = np.arange(5) % 3 - 1
    R0 = c3.cascade3_gemm(P["A"], P["B"], P["C"], kc=32)
    Ar = tuple(np.ldexp(x, r[:, None]) for x in P["A"])
    Bs = tuple(np.ldexp(x, s[None, :]) for x in P["B"])
    sh = r[:, None] + s[None, :]
    Cs = tuple(np.ldexp(x, sh) for x in P["C"])
    R1 = c3.cascade3_gemm(Ar, Bs, Cs, kc=32)
    for w in range(3):
        assert np.array_equal(R1[w], np.ldexp(R0[w], sh))


def test_k_zero_returns_C():
    P = make_problem3(3, 4, 0, cfg=7)
    R = c3.cascade3_gemm(P["A"], P["B"], P["C"])
    assert all(np.array_equal(R[w], P["C"][w]) for w in range(3))
