"""Seeded synthetic FP64x2 operands.

This module only draws random numbers and lays them out; it holds none of the
cascade's arithmetic, so both the HIP path's tests and the CPU oracle can take
their inputs from here.

Workload recipes (Sec. 5.2, "uniformly random data" and "wide-range data"):

* ``uniform``: ``hi ~ U[-1, 1)`` and ``lo = (hi * 2**-53) * U[-1, 1)``, so the
  pair carries about 106 significant bits and ``|lo| < ulp(hi)``.
* ``scaled``: as ``uniform``, but every row of A and every column of B is
  first multiplied by ``2**e`` with ``e`` a uniform integer in ``[-30, 30]``;
  C is multiplied by ``2**(e_i + f_j)`` so that it lives on the same scale as
  the product.  Exercises the per-row and per-column exponents.
* ``wide``: the paper's wide-range data.  For every row of A and every
  column of B two decimal exponents are drawn uniformly from ``[-60, 20]``
  and each gets a random sign, giving the end points ``x = s1 10**e1`` and
  ``y = s2 10**e2``; the row (column) is then filled with ``U[min, max]``
  draws, and ``lo = (hi * 2**-53) * U[-1, 1)`` as above.  C is zero (the
  experiment forms A B alone).  Rows whose range straddles zero hold values
  of every magnitude below the larger end point.
* ``panels``: as ``uniform``, but the scale changes along the inner
  dimension: every run of ``panel`` inner indices of every row of A is
  multiplied by ``2**e`` and of every column of B by ``2**f``, e and f
  uniform integers in ``[-40, 40]`` drawn independently per (row, panel)
  and (panel, column); C is scaled by ``2**max_b(e_ib + f_bj)``.  One
  exponent per whole row or column then fits only the largest panel.
* ``skewed``: as ``uniform``, but column p of A is multiplied by ``2**s_p``
  and row p of B by ``2**-s_p``, s_p a uniform integer in ``[-40, 40]``
  per inner index: every product keeps its ``uniform`` size while the row
  and column maxima are set by the most skewed index.

All arrays are float64 in Fortran (column-major) order, matching the BLAS
layout of the C ABI.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = 230304353
VARIANTS = {"uniform": 0, "scaled": 1, "wide": 2, "panels": 3, "skewed": 4}


def _rng(cfg: int, variant: str, m: int, n: int, k: int, salt: int = 0):
    return np.random.default_rng(
        np.random.SeedSequence([SEED_ROOT, int(cfg), VARIANTS[variant],
                                int(m), int(n), int(k), int(salt)]))


def _pair(rng, shape):
    hi = np.asfortranarray(rng.uniform(-1.0, 1.0, size=shape))
    u = np.asfortranarray(rng.uniform(-1.0, 1.0, size=shape))
    lo = np.asfortranarray((hi * 2.0 ** -53) * u)
    return hi, lo


def make_problem(m: int, n: int, k: int, *, cfg: int = 0, variant: str = "uniform",
                 salt: int = 0, panel: int = 256):
    """Return ``dict(A=(hi, lo), B=(hi, lo), C=(hi, lo))`` with A m×k, B k×n, C m×n."""
    rng = _rng(cfg, variant, m, n, k, salt)
    if variant == "wide":
        return _wide(rng, m, n, k)
    Ahi = np.asfortranarray(rng.uniform(-1.0, 1.0, size=(m, k)))
    Au = np.asfortranarray(rng.uniform(-1.0, 1.0, size=(m, k)))
    Bhi = np.asfortranarray(rng.uniform(-1.0, 1.0, size=(k, n)))
    Bu = np.asfortranarray(rng.uniform(-1.0, 1.0, size=(k, n)))
    Chi = np.asfortranarray(rng.uniform(-1.0, 1.0, size=(m, n)))
    Cu = np.asfortranarray(rng.uniform(-1.0, 1.0, size=(m, n)))
    if variant == "scaled":
        eA = rng.integers(-30, 31, size=m)
        fB = rng.integers(-30, 31, size=n)
        Ahi *= np.ldexp(1.0, eA)[:, None]
        Bhi *= np.ldexp(1.0, fB)[None, :]
        Chi *= np.ldexp(1.0, eA[:, None] + fB[None, :])
    elif variant == "skewed":
        sp = rng.integers(-40, 41, size=k)
        Ahi *= np.ldexp(1.0, sp)[None, :]
        Bhi *= np.ldexp(1.0, -sp)[:, None]
    elif variant == "panels":
        nb = max(1, -(-k // panel))
        eA = rng.integers(-40, 41, size=(m, nb))
        fB = rng.integers(-40, 41, size=(nb, n))
        pan = np.arange(k) // panel
        Ahi *= np.ldexp(1.0, eA[:, pan])
        Bhi *= np.ldexp(1.0, fB[pan, :])
        top = np.max(eA[:, :, None] + fB[None, :, :], axis=1) if m and n else np.zeros((m, n), dtype=np.int64)
        Chi *= np.ldexp(1.0, top)
    Alo = np.asfortranarray((Ahi * 2.0 ** -53) * Au)
    Blo = np.asfortranarray((Bhi * 2.0 ** -53) * Bu)
    Clo = np.asfortranarray((Chi * 2.0 ** -53) * Cu)
    return {"A": (Ahi, Alo), "B": (Bhi, Blo), "C": (Chi, Clo)}


def _ranges(rng, count):
    """Per-vector end points ``(lo, hi)`` of the wide-range recipe."""
    e = rng.uniform(-60.0, 20.0, size=(count, 2))
    sgn = np.where(rng.uniform(size=(count, 2)) < 0.5, -1.0, 1.0)
    ends = sgn * 10.0 ** e
    return ends.min(axis=1), ends.max(axis=1)


def _wide(rng, m, n, k):
    a0, a1 = _ranges(rng, m)
    b0, b1 = _ranges(rng, n)
    Ahi = np.asfortranarray(a0[:, None] + (a1 - a0)[:, None] * rng.uniform(size=(m, k)))
    Bhi = np.asfortranarray(b0[None, :] + (b1 - b0)[None, :] * rng.uniform(size=(k, n)))
    Alo = np.asfortranarray((Ahi * 2.0 ** -53) * rng.uniform(-1.0, 1.0, size=(m, k)))
    Blo = np.asfortranarray((Bhi * 2.0 ** -53) * rng.uniform(-1.0, 1.0, size=(k, n)))
    Z = np.zeros((m, n), order="F")
    return {"A": (Ahi, Alo), "B": (Bhi, Blo), "C": (Z, Z.copy()),
            "ranges": {"A": (a0, a1), "B": (b0, b1)}}


def make_problem3(m: int, n: int, k: int, *, cfg: int = 0, variant: str = "uniform", salt: int = 0):
    """FP64x3 operands: ``dict(A=(x0, x1, x2), B=..., C=...)`` with
    ``x0 ~ U[-1, 1)``, ``x1 = (x0 2**-53) U[-1, 1)``, ``x2 = (x1 2**-53) U[-1, 1)``
    (about 159 significant bits); ``scaled`` multiplies rows of A and columns
    of B (and C accordingly) by ``2**e``, e uniform in [-30, 30]."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 33, int(cfg), VARIANTS[variant],
                                                        int(m), int(n), int(k), int(salt)]))

    def words(shape):
        x0 = rng.uniform(-1.0, 1.0, size=shape)
        x1 = (x0 * 2.0 ** -53) * rng.uniform(-1.0, 1.0, size=shape)
        x2 = (x1 * 2.0 ** -53) * rng.uniform(-1.0, 1.0, size=shape)
        return [x0, x1, x2]

    A, B, C = words((m, k)), words((k, n)), words((m, n))
    if variant == "scaled":
        eA = rng.integers(-30, 31, size=m)
        fB = rng.integers(-30, 31, size=n)
        A = [x * np.ldexp(1.0, eA)[:, None] for x in A]
        B = [x * np.ldexp(1.0, fB)[None, :] for x in B]
        C = [x * np.ldexp(1.0, eA[:, None] + fB[None, :]) for x in C]
    elif variant != "uniform":
        raise ValueError("FP64x3 operands: uniform or scaled")
    f = lambda ws: tuple(np.asfortranarray(x) for x in ws)
    return {"A": f(A), "B": f(B), "C": f(C)}


def make_pair(shape, *, seed: int):
    """A single FP64x2 matrix of the ``uniform`` recipe (used by the autograd chain)."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 99, int(seed)] + list(shape)))
    return _pair(rng, tuple(shape))


def batched_shapes(count: int = 512, lo: int = 32, hi: int = 1024, *, seed: int = 3):
    """Shapes of the uneven batch: m, n, k each ``round(exp(U[ln lo, ln hi]))``."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 3, int(seed), count]))
    draw = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, 3)))).astype(np.int64)
    return [tuple(int(v) for v in row) for row in draw]


def sample_entries(m: int, n: int, count: int, *, seed: int = 7):
    """Seeded (i, j) output positions for sampled checks at full size."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 5, int(seed), m, n, count]))
    return rng.integers(0, m, size=count), rng.integers(0, n, size=count)
