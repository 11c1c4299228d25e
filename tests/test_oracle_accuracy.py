"""Pins of the accuracy-workload infrastructure (CPU only).

* the exact reference (expansion arithmetic) against rational arithmetic,
  including the wide-range and ill-conditioned inputs;
* the FP64x2 helpers of the ill-conditioned generator against rationals;
* the Householder QR: Q orthonormal and Q^T X upper triangular, exactly up to
  FP64x2 rounding;
* the ill-conditioned workload: A B equals the small target, one 1 per
  column, entries of magnitude in (t, 10 t), condition numbers near 1/t
  (eq. condnum);
* the wide-range recipe: per-vector ranges from decimal exponents in
  [-60, 20], every entry inside its range;
* the oracles' own errors on these workloads against the exact reference:
  the cascade within the FP64x2 tolerance, and more accurate than the
  FP64x2 triple loop on most entries of the ill-conditioned problems
  (the finding of Sec. 5.2).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import illcond as ic
from oracle.cascade import cascade_gemm
from oracle.ref import dd_gemm_ref, exact_entries
from oracle.slices import slices_gemm
from paper_2303_04353_amd.inputs import make_problem
from tests.exact import dd_value, exact_gemm

pytestmark = pytest.mark.filterwarnings("ignore")
F = Fraction


def _all(m, n):
    I, J = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    return I.ravel(), J.ravel()


def _workloads():
    yield "uniform", make_problem(7, 6, 33, cfg=120)
    yield "scaled", make_problem(6, 5, 40, cfg=121, variant="scaled")
    yield "wide", make_problem(8, 7, 30, cfg=122, variant="wide")
    W = ic.ill_conditioned(10, 1e-19, seed=4)
    yield "ill", W


@pytest.mark.parametrize("name,P", list(_workloads()), ids=lambda v: v if isinstance(v, str) else "")
def test_exact_entries_match_rationals(name, P):
    A, B, C = P["A"], P["B"], P["C"]
    m, n = C[0].shape
    I, J = _all(m, n)
    X = exact_gemm(A, B, C)
    R = dd_gemm_ref(A, B, C)[:2]
    ex, err = exact_entries(A, B, C, I, J, (R[0][I, J], R[1][I, J]))
    got = dd_value(R[0], R[1])
    for t, (i, j) in enumerate(zip(I, J)):
        V = X[i, j]
        D = got[i, j] - V
        # each output is the double nearest (to within one ulp) its exact value
        assert abs(F(ex[t]) - V) <= abs(V) * F(1, 2 ** 52), (name, i, j)
        assert abs(F(err[t]) - D) <= abs(D) * F(1, 2 ** 52), (name, i, j)


def test_exact_entries_sees_a_planted_error():
    P = make_problem(4, 3, 9, cfg=123)
    I, J = _all(4, 3)
    X = exact_gemm(P["A"], P["B"], P["C"])
    R = dd_gemm_ref(P["A"], P["B"], P["C"])[:2]
    Rh, Rl = R[0][I, J].copy(), R[1][I, J].copy()
    Rl[5] += 2.0 ** -80
    _, err = exact_entries(P["A"], P["B"], P["C"], I, J, (Rh, Rl))
    i, j = I[5], J[5]
    expect = F(float(Rh[5])) + F(float(Rl[5])) - X[i, j]
    assert abs(F(err[5]) - expect) <= abs(expect) * F(1, 2 ** 52)
    assert abs(err[5]) > 2.0 ** -82


def test_exact_entries_cancellation_to_zero_and_long_range():
    # x.y = 0 exactly with terms of very different sizes: the expansion keeps
    # every bit, the result is exactly zero
    big, small = 2.0 ** 300, 2.0 ** -300
    A = (np.array([[big, small, -big, -small]], order="F"), np.zeros((1, 4), order="F"))
    B = (np.array([[1.0], [1.0], [1.0], [1.0]], order="F"), np.zeros((4, 1), order="F"))
    C = (np.zeros((1, 1), order="F"), np.zeros((1, 1), order="F"))
    ex, err = exact_entries(A, B, C, np.array([0]), np.array([0]), (np.array([1.0]), np.array([0.0])))
    assert ex[0] == 0.0 and err[0] == 1.0
    A[0][0, 3] = 0.0   # leaves 2^-300 beside 2^300 - 2^300
    ex, _ = exact_entries(A, B, C, np.array([0]), np.array([0]), (np.array([0.0]), np.array([0.0])))
    assert ex[0] == small


# --- FP64x2 helpers of the generator -------------------------------------------

def _dd_rand(rng, n, scale=1.0):
    h = rng.uniform(0.5, 2.0, n) * scale * np.where(rng.uniform(size=n) < 0.5, -1, 1)
    l = h * 2.0 ** -53 * rng.uniform(-1, 1, n)
    return h, l


def _val(x, t):
    return F(float(x[0][t])) + F(float(x[1][t]))


def test_dd_helpers_against_rationals():
    rng = np.random.default_rng(5)
    n = 200
    x, y = _dd_rand(rng, n), _dd_rand(rng, n, 3.0)
    xp = (np.abs(x[0]), np.where(x[0] < 0, -x[1], x[1]))
    add, mul, div, sq = ic.dd_add(x, y), ic.dd_mul(x, y), ic.dd_div(x, y), ic.dd_sqrt(xp)
    u = F(1, 2 ** 100)
    for t in range(n):
        X, Y = _val(x, t), _val(y, t)
        assert abs(_val(add, t) - (X + Y)) <= u * (abs(X) + abs(Y))
        assert abs(_val(mul, t) - X * Y) <= u * abs(X * Y)
        assert abs(_val(div, t) - X / Y) <= u * abs(X / Y)
        s = _val(sq, t)
        # s^2 against |x| (exact square root is irrational in general)
        assert abs(s * s - abs(X)) <= 2 * u * abs(X)
    # the pairs come out normalised: |lo| <= ulp(hi) / 2
    for r in (add, mul, div, sq):
        assert np.all(np.abs(r[1]) <= np.abs(np.spacing(r[0])) / 2)


def test_dd_sum0_against_rationals():
    rng = np.random.default_rng(6)
    x = _dd_rand(rng, 37)
    h, l = ic.dd_sum0((x[0][:, None], x[1][:, None]))
    S = sum(_val(x, t) for t in range(37))
    A = sum(abs(_val(x, t)) for t in range(37))
    assert abs(F(float(h[0])) + F(float(l[0])) - S) <= 37 * F(1, 2 ** 100) * A


# --- Householder QR in FP64x2 ---------------------------------------------------

def test_householder_q_is_orthonormal_and_triangularises_exactly():
    rng = np.random.default_rng(7)
    n = 9
    X = rng.uniform(-1, 1, (n, n))
    Qh, Ql = ic.householder_q(X)
    Q = dd_value(Qh, Ql)
    tol = F(1, 10 ** 29)
    for i in range(n):
        for j in range(n):
            g = sum(Q[i, p] * Q[j, p] for p in range(n))
            assert abs(g - (1 if i == j else 0)) <= tol, (i, j)
            # (Q^T X)_ij below the diagonal vanishes: X = Q R
            if i > j:
                r = sum(Q[p, i] * F(float(X[p, j])) for p in range(n))
                assert abs(r) <= tol, (i, j)


def test_householder_q_orthonormal_at_size():
    rng = np.random.default_rng(8)
    n = 96
    Qh, Ql = ic.householder_q(rng.uniform(-1, 1, (n, n)))
    G = dd_gemm_ref((Qh, Ql), (Qh, Ql), transb=True)
    E = (G[0] - np.eye(n)) + G[1]
    assert np.max(np.abs(E)) < 1e-29


# --- the ill-conditioned workload -----------------------------------------------

@pytest.mark.parametrize("t", [1e-9, 1e-14, 1e-19])
def test_ill_conditioned_structure(t):
    n = 12
    W = ic.ill_conditioned(n, t, seed=2)
    T = W["target"]
    ones = T == 1.0
    assert np.all(ones.sum(axis=0) == 1)
    mag = np.abs(T[~ones])
    assert np.all(mag > t) and np.all(mag < 10 * t)
    assert np.all(W["C"][0] == 0) and np.all(W["C"][1] == 0)
    # A B = T up to FP64x2 rounding of Q and of B = Q^T T
    X = exact_gemm(W["A"], W["B"])
    for i in range(n):
        for j in range(n):
            assert abs(X[i, j] - F(float(T[i, j]))) <= F(1, 10 ** 29), (i, j)
    # unit rows of A, columns of B of norm about one: condition about 1/|T_ij|
    rn = np.sqrt(np.sum(W["A"][0] ** 2, axis=1))
    cn = np.sqrt(np.sum(W["B"][0] ** 2, axis=0))
    assert np.allclose(rn, 1.0, rtol=1e-14) and np.all((cn > 0.99) & (cn < 1.01 + 10 * n * t))
    cond = rn[:, None] * cn[None, :] / np.abs(T)
    assert np.all(cond[~ones] > 0.09 / t)


def test_ill_conditioned_is_seeded():
    a = ic.ill_conditioned(8, 1e-14, seed=3)
    b = ic.ill_conditioned(8, 1e-14, seed=3)
    c = ic.ill_conditioned(8, 1e-14, seed=4)
    assert np.array_equal(a["B"][0], b["B"][0]) and np.array_equal(a["B"][1], b["B"][1])
    assert not np.array_equal(a["B"][0], c["B"][0])


# --- the wide-range recipe --------------------------------------------------------

def test_wide_range_recipe():
    m, n, k = 300, 250, 20
    P = make_problem(m, n, k, cfg=124, variant="wide")
    (a0, a1), (b0, b1) = P["ranges"]["A"], P["ranges"]["B"]
    for lo, hi in ((a0, a1), (b0, b1)):
        assert np.all(lo <= hi)
        for e in (lo, hi):
            d = np.log10(np.abs(e))
            assert np.all((d >= -60 - 1e-9) & (d <= 20 + 1e-9))
        # every sign pattern of the end points occurs
        assert np.any(lo < 0) and np.any(hi > 0) and np.any(lo > 0) and np.any(hi < 0)
    Ah, Bh = P["A"][0], P["B"][0]
    assert np.all((Ah >= a0[:, None]) & (Ah <= a1[:, None]))
    assert np.all((Bh >= b0[None, :]) & (Bh <= b1[None, :]))
    assert np.all(np.abs(P["A"][1]) <= np.abs(Ah) * 2.0 ** -53)
    # magnitudes really vary from vector to vector: over 60 decades
    amax = np.log10(np.max(np.abs(Ah), axis=1))
    assert amax.max() - amax.min() > 60
    assert np.all(P["C"][0] == 0)


# --- the oracles on the paper's accuracy workloads -----------------------------

def _errors(P, R):
    m, n = P["C"][0].shape
    I, J = _all(m, n)
    ex, err = exact_entries(P["A"], P["B"], P["C"], I, J, (R[0][I, J], R[1][I, J]))
    return ex, err, I, J


@pytest.mark.parametrize("t", [1e-9, 1e-14, 1e-19])
def test_cascade_beats_fp64x2_on_ill_conditioned_products(t):
    n = 64
    W = ic.ill_conditioned(n, t, seed=5)
    D = dd_gemm_ref(W["A"], W["B"], W["C"])[:2]
    G = cascade_gemm(W["A"], W["B"], W["C"])
    S = slices_gemm(W["A"], W["B"], W["C"])
    ex, ed, I, J = _errors(W, D)
    _, eg, _, _ = _errors(W, G)
    _, es, _, _ = _errors(W, S)
    AB = np.abs(W["A"][0]) @ np.abs(W["B"][0])
    tol = 64 * n * 2.0 ** -104 * AB[I, J]
    assert np.all(np.abs(eg) <= tol) and np.all(np.abs(es) <= tol)
    assert np.all(np.abs(ed) <= tol)
    # componentwise relative errors: the cascade wins on most entries
    rd, rg = np.abs(ed) / np.abs(ex), np.abs(eg) / np.abs(ex)
    assert np.mean(rg <= rd) > 0.9
    assert np.median(rd / np.maximum(rg, 1e-300)) > 10
    # the errors grow with the conditioning: relative error about cond * 2^-106
    assert rd.max() > 0.01 * 2.0 ** -106 / t


def test_cascade_on_wide_range_inputs():
    P = make_problem(48, 40, 64, cfg=125, variant="wide")
    D = dd_gemm_ref(P["A"], P["B"], P["C"])[:2]
    G = cascade_gemm(P["A"], P["B"], P["C"])
    ex, ed, I, J = _errors(P, D)
    _, eg, _, _ = _errors(P, G)
    AB = np.abs(P["A"][0]) @ np.abs(P["B"][0])
    tol = 64 * 64 * 2.0 ** -104 * AB[I, J]
    assert np.all(np.abs(eg) <= tol) and np.all(np.abs(ed) <= tol)
    assert np.mean(np.abs(eg) <= np.abs(ed)) > 0.9


# --- Sec. 3.6 discussion (eq. fp642err): a nonzero bin 0 bounds the error ------------

@pytest.mark.parametrize("name", ["ill-1e-14", "ill-1e-19", "wide", "uniform"])
def test_nonzero_bin0_bounds_the_relative_error(name):
    # With one rank-kc block (k <= kc): a nonzero bin 0 needs a product of two
    # nonzero leading digits, i.e. |x_p| >= 2^-c0 sigma and |y_p| >= 2^-c0 tau
    # (rounding to the grid 2^(1-c0) gives 0 below half a grid step), so
    # |x|^T |y| >= 2^-(2 c0 + 2) ||x|| ||y||.  Put into eq. (cascerr), the error
    # is then at most (2^-106 + 40 k kc eps~ 2^(2 c0 + 2)) |x|^T |y|.
    n = 64
    P = ic.ill_conditioned(n, float(name[4:]), seed=6) if name.startswith("ill") else \
        make_problem(n, n, n, cfg=126, variant=name)
    hi, lo, parts = cascade_gemm(P["A"], P["B"], P["C"], kc=256, return_parts=True)
    assert len(parts["bins"]) == 1
    bin0 = parts["bins"][0][0]
    c0 = parts["c"][0]
    eps_t = 2.0 ** -(sum(parts["c"]) + 53)
    ex, err, I, J = _errors(P, (hi, lo))
    absx_absy = (np.abs(P["A"][0]) @ np.abs(P["B"][0]))[I, J]
    xinf = np.max(np.abs(P["A"][0]), axis=1)[I]
    yinf = np.max(np.abs(P["B"][0]), axis=0)[J]
    nz = bin0[I, J] != 0
    assert np.mean(nz) > 0.5
    # the lower bound, with a margin for the FP64 evaluation of |x|^T |y|
    assert np.all(absx_absy[nz] >= (1 - 1e-12) * 2.0 ** -(2 * c0 + 2) * xinf[nz] * yinf[nz])
    bound = (2.0 ** -106 + 40 * n * n * eps_t * 2.0 ** (2 * c0 + 2)) * absx_absy
    C = np.abs(P["C"][0][I, J])
    assert np.all(np.abs(err[nz]) <= bound[nz] + 2.0 ** -104 * C[nz])
