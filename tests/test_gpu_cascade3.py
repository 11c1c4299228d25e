"""GPU parity of the FP64x3 cascade (C ABI ``td_gemm_ex``) against the oracle.

Bins 0..4 are exact on both sides and the split, the triple-word sums and
the epilogue are the same fixed sequences of round-to-nearest operations,
so the results may differ only through the order in which the library and
numpy sum the tail bin; the bound below covers that.  Also: exact rationals
on a small problem, integer matrices, transposed storage, k = 0, non-finite
entries (NaN only in their rows and columns), padded leading dimensions.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import cascade3 as c3
from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import make_problem3
from tests.gpuhelp import down, log, up

pytestmark = pytest.mark.gpu


def run_td(A, B, C, *, transa=False, transb=False, kc=0):
    import torch
    m = A[0].shape[1] if transa else A[0].shape[0]
    k = A[0].shape[0] if transa else A[0].shape[1]
    n = B[0].shape[0] if transb else B[0].shape[1]
    Ad = [up(x) for x in A]
    Bd = [up(x) for x in B]
    Cd = [up(x) for x in C]
    st = dg.td_gemm_ex(int(transa), int(transb), m, n, k, *Ad, max(1, A[0].shape[0]), *Bd, max(1, B[0].shape[0]),
                       *Cd, max(1, C[0].shape[0]), kc=kc)
    dg.check(st, "td_gemm_ex")
    torch.cuda.synchronize()
    return tuple(down(x) for x in Cd)


def _diff(G, O):
    return np.abs(((G[0] - O[0]) + (G[1] - O[1])) + (G[2] - O[2]))


def _order_bound(A, B, O, k, kc):
    kce = min(kc, k)
    D4 = sum(c3.widths3(kce))
    e = c3.exponents(A[0], axis=1).astype(np.int64)
    f = c3.exponents(B[0], axis=0).astype(np.int64)
    nb = -(-k // kce)
    AB = np.abs(A[0]) @ np.abs(B[0])
    return (np.ldexp(1.0, e[:, None] + f[None, :]) * nb * 1024.0 * kce * kce * 2.0 ** -(53 + D4)
            + 2.0 ** -150 * (np.abs(O[0]) + AB))


CASES = [(64, 64, 64, 256, "uniform"), (100, 70, 300, 256, "uniform"), (65, 33, 17, 256, "scaled"),
         (1, 1, 1, 256, "uniform"), (130, 96, 520, 128, "scaled"), (40, 50, 1000, 64, "uniform")]


@pytest.mark.parametrize("m,n,k,kc,variant", CASES)
def test_td_matches_the_oracle(m, n, k, kc, variant):
    log(f"td m={m} n={n} k={k} kc={kc} {variant}")
    P = make_problem3(m, n, k, cfg=30, variant=variant)
    G = run_td(P["A"], P["B"], P["C"], kc=kc)
    O = c3.cascade3_gemm(P["A"], P["B"], P["C"], kc=kc)
    assert np.all(_diff(G, O) <= _order_bound(P["A"], P["B"], O, k, kc))
    # the words come out renormalised: each within the previous word's ulp
    assert np.all(np.abs(G[1]) <= np.spacing(np.abs(G[0]))) and np.all(np.abs(G[2]) <= np.spacing(np.abs(G[1])) + 1e-300)


def test_td_long_inner_dimension():
    """k = 20003: 79 rank-256 blocks (the last one of 35 indices), each added
    to the triple-word accumulator."""
    m, n, k = 40, 24, 20003
    log(f"td long k: m={m} n={n} k={k}")
    P = make_problem3(m, n, k, cfg=9)
    G = run_td(P["A"], P["B"], P["C"])
    O = c3.cascade3_gemm(P["A"], P["B"], P["C"], kc=256)
    assert np.all(_diff(G, O) <= _order_bound(P["A"], P["B"], O, k, 256))


@pytest.mark.parametrize("kc", [12, 20, 28])
def test_td_blocks_ending_mid_iteration(kc):
    """kc / 4 = 3, 5, 7 groups per block: the combines fall at every position
    of the product loop's six-group iteration and of its tail."""
    m, n, k = 40, 70, 230
    log(f"td kc={kc} m={m} n={n} k={k}")
    P = make_problem3(m, n, k, cfg=10)
    G = run_td(P["A"], P["B"], P["C"], kc=kc)
    O = c3.cascade3_gemm(P["A"], P["B"], P["C"], kc=kc)
    assert np.all(_diff(G, O) <= _order_bound(P["A"], P["B"], O, k, kc))


def test_td_against_exact_rationals():
    m, n, k = 4, 3, 40
    P = make_problem3(m, n, k, cfg=31)
    G = run_td(P["A"], P["B"], P["C"], kc=16)
    val = lambda ws, idx: sum(Fraction(float(w[idx])) for w in ws)
    for i in range(m):
        for j in range(n):
            X = sum(val(P["A"], (i, p)) * val(P["B"], (p, j)) for p in range(k)) + val(P["C"], (i, j))
            S = sum(abs(val(P["A"], (i, p)) * val(P["B"], (p, j))) for p in range(k))
            assert abs(val(G, (i, j)) - X) <= Fraction(1, 2 ** 150) * (S + abs(X)), (i, j)


def test_td_integer_matrices_exact_and_transposes():
    rng = np.random.default_rng(32)
    m, n, k = 70, 50, 700
    A = np.asfortranarray(rng.integers(-2 ** 20, 2 ** 20 + 1, size=(m, k)).astype(float))
    B = np.asfortranarray(rng.integers(-2 ** 20, 2 ** 20 + 1, size=(k, n)).astype(float))
    z = lambda s: np.zeros(s, order="F")
    G = run_td((A, z(A.shape), z(A.shape)), (B, z(B.shape), z(B.shape)), (z((m, n)), z((m, n)), z((m, n))))
    want = A.astype(object) @ B.astype(object)
    assert np.all(G[0].astype(object) == want) and np.all(G[1] == 0) and np.all(G[2] == 0)
    P = make_problem3(70, 90, 333, cfg=33)
    G0 = run_td(P["A"], P["B"], P["C"])
    At = tuple(np.asfortranarray(x.T) for x in P["A"])
    Bt = tuple(np.asfortranarray(x.T) for x in P["B"])
    G1 = run_td(At, Bt, P["C"], transa=True, transb=True)
    assert all(np.array_equal(G0[w], G1[w]) for w in range(3))
    G2 = run_td(At, P["B"], P["C"], transa=True)
    G3 = run_td(P["A"], Bt, P["C"], transb=True)
    assert all(np.array_equal(G0[w], G2[w]) and np.array_equal(G0[w], G3[w]) for w in range(3))


def test_td_k_zero_leaves_C():
    P = make_problem3(9, 7, 0, cfg=34)
    G = run_td(P["A"], P["B"], P["C"])
    assert all(np.array_equal(G[w], P["C"][w]) for w in range(3))


def test_td_non_finite_rows_and_columns_become_nan_only_there():
    m, n, k = 20, 12, 40
    P = make_problem3(m, n, k, cfg=35)
    A = tuple(x.copy(order="F") for x in P["A"])
    B = tuple(x.copy(order="F") for x in P["B"])
    A[0][3, 7] = np.inf        # leading word
    A[2][11, 2] = np.nan       # third word of a finite leading word
    B[1][5, 4] = -np.inf       # second word of a column of B
    G = run_td(A, B, P["C"], kc=16)
    badr = np.zeros(m, bool)
    badr[[3, 11]] = True
    badc = np.zeros(n, bool)
    badc[4] = True
    bad = badr[:, None] | badc[None, :]
    assert np.all(np.isnan(G[0][bad]))
    assert all(np.all(np.isfinite(G[w][~bad])) for w in range(3))
    Af = tuple(x[~badr] for x in A)
    Bf = tuple(x[:, ~badc] for x in B)
    Cf = tuple(x[~badr][:, ~badc] for x in P["C"])
    O = c3.cascade3_gemm(Af, Bf, Cf, kc=16)
    Gf = tuple(x[~badr][:, ~badc] for x in G)
    assert np.all(_diff(Gf, O) <= _order_bound(Af, Bf, O, k, 16))


def test_td_padded_leading_dimensions_bit_identical():
    import torch
    m, n, k = 37, 29, 300
    P = make_problem3(m, n, k, cfg=36)
    G0 = run_td(P["A"], P["B"], P["C"])
    lda, ldb, ldc = m + 3, k + 5, m + 2
    def pad(x, ld):
        out = np.full((ld, x.shape[1]), 7.0, order="F")
        out[:x.shape[0]] = x
        return out
    Ad = [up(pad(x, lda)) for x in P["A"]]
    Bd = [up(pad(x, ldb)) for x in P["B"]]
    Cd = [up(pad(x, ldc)) for x in P["C"]]
    dg.check(dg.td_gemm_ex(0, 0, m, n, k, *Ad, lda, *Bd, ldb, *Cd, ldc), "td_gemm_ex")
    torch.cuda.synchronize()
    G1 = [down(x) for x in Cd]
    for w in range(3):
        assert np.array_equal(G1[w][:m], G0[w])
        assert np.all(G1[w][m:] == 7.0)   # rows beyond m untouched
