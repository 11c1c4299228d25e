"""Pins of the plain FP64x2 triple-loop oracle (CPU only).

Against: exact rational arithmetic, integer matrices, identity/permutation,
k = 0, sign and power-of-two symmetry, cancellation with a representable
result, transposition.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle.ref import dd_gemm_ref, dd_gemm_ref_entries, max_threads
from paper_2303_04353_amd.inputs import make_problem
from tests.exact import abs_gemm, dd_value, exact_gemm

pytestmark = pytest.mark.filterwarnings("ignore")
U2 = Fraction(1, 2 ** 106)  # FP64x2 unit roundoff


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 2, 2), (5, 4, 17), (6, 6, 6), (2, 7, 1)])
def test_matches_exact_rationals(m, n, k):
    P = make_problem(m, n, k, cfg=90)
    hi, lo, _ = dd_gemm_ref(P["A"], P["B"], P["C"])
    X = exact_gemm(P["A"], P["B"], P["C"])
    S = abs_gemm(P["A"], P["B"]) + np.abs(dd_value(*P["C"]))
    got = dd_value(hi, lo)
    for idx in np.ndindex(X.shape):
        err = abs(got[idx] - X[idx])
        assert err <= (3 * k + 8) * U2 * S[idx], (idx, float(err), float(S[idx]))


def test_integer_matrices_exact():
    rng = np.random.default_rng(1)
    m, n, k = 9, 7, 4096
    A = rng.integers(-2 ** 20, 2 ** 20 + 1, size=(m, k))
    B = rng.integers(-2 ** 20, 2 ** 20 + 1, size=(k, n))
    C = rng.integers(-2 ** 40, 2 ** 40 + 1, size=(m, n))
    # |sum| <= 4096 * 2^40 + 2^40 < 2^53: every partial sum is an exact FP64 integer
    z = lambda s: np.zeros(s)
    hi, lo, _ = dd_gemm_ref((A.astype(float), z(A.shape)), (B.astype(float), z(B.shape)),
                            (C.astype(float), z(C.shape)))
    want = A.astype(object) @ B.astype(object) + C.astype(object)
    assert np.all(hi.astype(object) == want)
    assert np.all(lo == 0.0)


def test_identity_and_permutation_exact():
    n, k = 5, 6
    P = make_problem(k, n, k, cfg=91)
    B = P["B"]
    I = (np.eye(k), np.zeros((k, k)))
    hi, lo, _ = dd_gemm_ref(I, B)
    assert np.all(dd_value(hi, lo) == dd_value(*B))
    perm = np.array([3, 0, 5, 1, 4, 2])
    Pm = np.eye(k)[perm]
    hi, lo, _ = dd_gemm_ref((Pm, np.zeros((k, k))), B)
    assert np.all(dd_value(hi, lo) == dd_value(B[0][perm], B[1][perm]))


def test_k_zero_leaves_c_bitwise():
    P = make_problem(4, 3, 0, cfg=92)
    Chi, Clo = P["C"]
    hi, lo, _ = dd_gemm_ref(P["A"], P["B"], P["C"])
    assert np.array_equal(hi, Chi) and np.array_equal(lo, Clo)


def test_sign_and_power_of_two_symmetry_bitwise():
    P = make_problem(8, 6, 33, cfg=93)
    A, B = P["A"], P["B"]
    h0, l0, _ = dd_gemm_ref(A, B)
    h1, l1, _ = dd_gemm_ref((-A[0], -A[1]), B)
    assert np.array_equal(h1, -h0) and np.array_equal(l1, -l0)
    h2, l2, _ = dd_gemm_ref((A[0] * 2.0 ** 37, A[1] * 2.0 ** 37), (B[0] * 2.0 ** -11, B[1] * 2.0 ** -11))
    assert np.array_equal(h2, h0 * 2.0 ** 26) and np.array_equal(l2, l0 * 2.0 ** 26)


def test_cancellation_with_representable_result_is_exact():
    # (1 + 2^-60) * 1 + (-1 + 3*2^-120) * 1 = 2^-60 + 3*2^-120 exactly; the low
    # words only survive if the DD addition keeps the error of lo + lo.
    A = (np.array([[1.0, -1.0]]), np.array([[2.0 ** -60, 3 * 2.0 ** -120]]))
    B = (np.array([[1.0], [1.0]]), np.zeros((2, 1)))
    hi, lo, _ = dd_gemm_ref(A, B)
    assert hi[0, 0] == 2.0 ** -60 and lo[0, 0] == 3 * 2.0 ** -120
    # the cross terms of the DD product: (1 + 2^-60)(1 + 2^-70) has the
    # representable value 1 + 2^-60 + 2^-70 (+ 2^-130, below the FP64x2 grid)
    A = (np.array([[1.0]]), np.array([[2.0 ** -60]]))
    B = (np.array([[1.0]]), np.array([[2.0 ** -70]]))
    hi, lo, _ = dd_gemm_ref(A, B)
    assert hi[0, 0] == 1.0 and lo[0, 0] == 2.0 ** -60 + 2.0 ** -70


def test_transposes_agree_bitwise():
    P = make_problem(7, 5, 19, cfg=94)
    A, B, C = P["A"], P["B"], P["C"]
    h0, l0, _ = dd_gemm_ref(A, B, C)
    At = (np.asfortranarray(A[0].T), np.asfortranarray(A[1].T))
    Bt = (np.asfortranarray(B[0].T), np.asfortranarray(B[1].T))
    h1, l1, _ = dd_gemm_ref(At, Bt, C, transa=True, transb=True)
    assert np.array_equal(h0, h1) and np.array_equal(l0, l1)
    h2, l2, _ = dd_gemm_ref(At, B, C, transa=True)
    assert np.array_equal(h0, h2) and np.array_equal(l0, l2)


def test_entries_equal_full_bitwise_and_threads():
    P = make_problem(20, 13, 40, cfg=95)
    h0, l0, used = dd_gemm_ref(P["A"], P["B"], P["C"])
    assert 1 <= used <= max(1, max_threads())
    I = np.array([0, 19, 7, 3, 3])
    J = np.array([0, 12, 5, 0, 11])
    h1, l1, _ = dd_gemm_ref_entries(P["A"], P["B"], P["C"], I, J)
    assert np.array_equal(h1, h0[I, J]) and np.array_equal(l1, l0[I, J])


def test_dd_add_vector_against_rationals():
    """The entry-wise accurate FP64x2 addition of the C oracle (the one its
    triple loop accumulates with).  When the high words cancel, the low
    words' error-free sum survives: (1, 2^-60) + (-1, 3 2^-114) is
    2^-60 + 3 2^-114 exactly, held as (2^-60 + 2^-112, -2^-114); two
    disjoint words add exactly; x + 0 = x; on random pairs with heavy
    cancellation the relative error is within 3 2^-106, the published bound
    of this algorithm (Joldes, Muller and Popescu, 2017: AccurateDWPlusDW),
    and the result is a normalised pair (|lo| <= ulp(hi) / 2)."""
    from oracle.ref import dd_add_ref
    h, l = dd_add_ref((np.array([1.0, 0.5, 0.75]), np.array([2.0 ** -60, 0.0, 2.0 ** -60])),
                      (np.array([-1.0, 2.0 ** -70, 0.0]), np.array([3 * 2.0 ** -114, 0.0, 0.0])))
    assert (float(h[0]), float(l[0])) == (2.0 ** -60 + 2.0 ** -112, -2.0 ** -114)
    assert (float(h[1]), float(l[1])) == (0.5, 2.0 ** -70)
    assert (float(h[2]), float(l[2])) == (0.75, 2.0 ** -60)
    rng = np.random.default_rng(81)
    n = 20000
    xh = rng.uniform(-1, 1, n) * np.ldexp(1.0, rng.integers(-20, 20, n))
    xl = xh * rng.uniform(-1, 1, n) * 2.0 ** -53
    yh = -xh * (1 + rng.integers(-8, 9, n) * 2.0 ** -52)
    yh[::3] = rng.uniform(-1, 1, (n + 2) // 3)            # and some without cancellation
    yl = yh * rng.uniform(-1, 1, n) * 2.0 ** -53
    # normalised pairs, as the bound assumes (QuickTwoSum: |hi| >= |lo|)
    qs = lambda a, b: (a + b, b - ((a + b) - a))
    (xh, xl), (yh, yl) = qs(xh, xl), qs(yh, yl)
    h, l = dd_add_ref((xh, xl), (yh, yl))
    for t in range(n):
        exact = Fraction(float(xh[t])) + Fraction(float(xl[t])) + Fraction(float(yh[t])) + Fraction(float(yl[t]))
        got = Fraction(float(h[t])) + Fraction(float(l[t]))
        assert abs(got - exact) <= 3 * U2 * abs(exact), t
        assert h[t] == 0 or abs(l[t]) <= np.spacing(abs(h[t])) / 2, t
