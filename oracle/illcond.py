"""TEST INFRASTRUCTURE: the paper's ill-conditioned GEMM workload (Sec. 5.2,
the ill-conditioned experiments).

A = Q with orthonormal rows, from the Householder QR of a seeded random
matrix computed in FP64x2 arithmetic (the paper uses quad precision); C has
entries of magnitude in (t, 10 t) with random signs and one entry equal to 1
in every column; B = Q^T C computed in FP64x2 (the oracle's triple loop).
Then every entry of A B = C is the dot product of a unit row of A with a
column of B of norm about 1, and all but one per column come out near t: dot
products with condition numbers about 1/t (eq. condnum).

Only the tests and the benchmark's CPU-baseline leg use this module.  The
FP64x2 arithmetic here (TwoSum; Dekker's TwoProduct with Veltkamp splitting,
so no fused multiply-add is needed in numpy; Newton steps for division and
square root) builds inputs; it is not the method under test.
"""
from __future__ import annotations

import numpy as np

from .cascade import quick_two_sum, two_sum
from .ref import dd_gemm_ref

_SPLIT = 134217729.0   # 2^27 + 1


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dd_add(x, y):
    s, e = two_sum(x[0], y[0])
    t, f = two_sum(x[1], y[1])
    e = e + t
    s, e = quick_two_sum(s, e)
    e = e + f
    return quick_two_sum(s, e)


def dd_mul(x, y):
    p, e = _two_prod(x[0], y[0])
    e = e + (x[0] * y[1] + x[1] * y[0])
    return quick_two_sum(p, e)


def dd_neg(x):
    return -x[0], -x[1]


def dd_div(x, y):
    q1 = x[0] / y[0]
    r = dd_add(x, dd_neg(dd_mul((q1, np.zeros_like(q1)), y)))
    q2 = r[0] / y[0]
    r = dd_add(r, dd_neg(dd_mul((q2, np.zeros_like(q2)), y)))
    q3 = r[0] / y[0]
    s, e = quick_two_sum(q1, q2)
    return dd_add((s, e), (q3, np.zeros_like(q3)))


def dd_sqrt(x):
    s = np.sqrt(x[0])
    # one Newton step in FP64x2: s + (x - s^2) / (2 s)
    s2 = dd_mul((s, np.zeros_like(s)), (s, np.zeros_like(s)))
    r = dd_add(x, dd_neg(s2))
    corr = r[0] / (2.0 * s)
    return quick_two_sum(s, corr)


def dd_sum0(x):
    """Sum over axis 0 in FP64x2 (pairwise tree)."""
    h, l = x
    while h.shape[0] > 1:
        n = h.shape[0]
        half = n // 2
        a = (h[:half], l[:half])
        b = (h[half:2 * half], l[half:2 * half])
        sh, sl = dd_add(a, b)
        if n % 2:
            sh = np.concatenate([sh, h[-1:]], axis=0)
            sl = np.concatenate([sl, l[-1:]], axis=0)
        h, l = sh, sl
    return h[0], l[0]


def householder_q(X):
    """Q of the Householder QR of the square FP64 matrix X, in FP64x2 (hi, lo)."""
    n = X.shape[0]
    Rh = np.array(X, dtype=np.float64)
    Rl = np.zeros_like(Rh)
    vs = []
    for j in range(n - 1):
        xh, xl = Rh[j:, j].copy(), Rl[j:, j].copy()
        nrm = dd_sqrt(dd_sum0(dd_mul((xh, xl), (xh, xl))))
        sign = 1.0 if xh[0] >= 0 else -1.0
        alpha = (-sign * nrm[0], -sign * nrm[1])
        vh, vl = xh.copy(), xl.copy()
        v0 = dd_add((np.array([xh[0]]), np.array([xl[0]])), (np.array([-alpha[0]]), np.array([-alpha[1]])))
        vh[0], vl[0] = v0[0][0], v0[1][0]
        vtv = dd_sum0(dd_mul((vh, vl), (vh, vl)))
        beta = dd_div((np.array([2.0]), np.array([0.0])), (np.array([vtv[0]]), np.array([vtv[1]])))
        beta = (beta[0][0], beta[1][0])
        vs.append((j, vh, vl, beta))
        # R[j:, j:] -= beta v (v^T R[j:, j:])
        sub = (Rh[j:, j:], Rl[j:, j:])
        w = dd_sum0(dd_mul((vh[:, None], vl[:, None]), sub))
        bw = dd_mul((beta[0], beta[1]), w)
        upd = dd_mul((vh[:, None], vl[:, None]), (bw[0][None, :], bw[1][None, :]))
        Rh[j:, j:], Rl[j:, j:] = dd_add(sub, dd_neg(upd))
    Qh = np.eye(n)
    Ql = np.zeros((n, n))
    for j, vh, vl, beta in reversed(vs):
        sub = (Qh[j:, :], Ql[j:, :])
        w = dd_sum0(dd_mul((vh[:, None], vl[:, None]), sub))
        bw = dd_mul((beta[0], beta[1]), w)
        upd = dd_mul((vh[:, None], vl[:, None]), (bw[0][None, :], bw[1][None, :]))
        Qh[j:, :], Ql[j:, :] = dd_add(sub, dd_neg(upd))
    return Qh, Ql


def ill_conditioned(n: int, t: float, *, seed: int = 0):
    """The ill-conditioned n x n x n workload for tolerance t: returns
    ``dict(A=(hi, lo), B=(hi, lo), C=(zeros), target=C_t)`` in Fortran order,
    C being the zero matrix the GEMM adds to and ``target`` the matrix of small
    entries that A B approximates."""
    rng = np.random.default_rng(np.random.SeedSequence([230304353, 77, int(n), int(seed), int(round(-np.log10(t)))]))
    X = rng.uniform(-1.0, 1.0, size=(n, n))
    Qh, Ql = householder_q(X)
    mag = rng.uniform(1.0, 10.0, size=(n, n)) * t
    sgn = np.where(rng.uniform(size=(n, n)) < 0.5, -1.0, 1.0)
    T = mag * sgn
    ones = rng.integers(0, n, size=n)
    T[ones, np.arange(n)] = 1.0
    A = (np.asfortranarray(Qh), np.asfortranarray(Ql))
    # B = Q^T T in FP64x2 (the oracle's triple loop, transposed first operand)
    Bh, Bl, _ = dd_gemm_ref(A, (np.asfortranarray(T), np.zeros((n, n), order="F")), transa=True)
    zeros = (np.zeros((n, n), order="F"), np.zeros((n, n), order="F"))
    return {"A": A, "B": (np.asfortranarray(Bh), np.asfortranarray(Bl)), "C": zeros,
            "target": np.asfortranarray(T)}
