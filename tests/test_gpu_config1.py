"""GPU checks of the square FP64x2 GEMMs at 1024^3 and 4096^3, uniform and
ill-scaled.

The ill-scaled problem is built from the uniform draws: row i of A and
column j of B (both words) times 2^e_i and 2^f_j, C times 2^(e_i + f_j), e
and f uniform integers in [-30, 30].  Every path takes its powers of two
from the row and column maxima and scales exactly, so the ill-scaled result
must be the uniform one times 2^(e_i + f_j), bit for bit.  Sampled entries
of the ill-scaled result are held to the FP64x2 oracle's tolerance,
64 k 2^-104 (|A||B|)_ij.
"""
import numpy as np
import pytest

from oracle.ref import dd_gemm_ref_entries
from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import SEED_ROOT, make_problem, sample_entries
from tests.gpuhelp import log, run_gemm

pytestmark = pytest.mark.gpu

ALGOS = [("cascade", dg.DD_ALGO_CASCADE_F64), ("dd_valu", dg.DD_ALGO_DD_VALU),
         ("slices_bf16", dg.DD_ALGO_SLICES_BF16), ("slices_i8", dg.DD_ALGO_SLICES_I8)]


def _ill_scaled(P, size):
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, 1, 17, size]))
    e = rng.integers(-30, 31, size=size)
    f = rng.integers(-30, 31, size=size)
    sa, sb, sc = np.ldexp(1.0, e)[:, None], np.ldexp(1.0, f)[None, :], np.ldexp(1.0, e[:, None] + f[None, :])
    S = {"A": tuple(np.asfortranarray(x * sa) for x in P["A"]),
         "B": tuple(np.asfortranarray(x * sb) for x in P["B"]),
         "C": tuple(np.asfortranarray(x * sc) for x in P["C"])}
    return S, sc


@pytest.mark.parametrize("size", [1024, 4096])
def test_ill_scaled_equals_uniform_times_powers_of_two(size):
    P = make_problem(size, size, size, cfg=1)
    S, sc = _ill_scaled(P, size)
    I, J = sample_entries(size, size, 256, seed=size)
    rh, rl, _ = dd_gemm_ref_entries(S["A"], S["B"], S["C"], I, J)
    AB = np.array([np.abs(S["A"][0][i]) @ np.abs(S["B"][0][:, j]) for i, j in zip(I, J)])
    tol = 64 * size * 2.0 ** -104 * AB
    for name, algo in ALGOS:
        log(f"config 1 {size}^3 {name}: uniform and ill-scaled")
        Gu = run_gemm(P["A"], P["B"], P["C"], algo=algo)
        Gs = run_gemm(S["A"], S["B"], S["C"], algo=algo)
        assert np.array_equal(Gs[0], Gu[0] * sc) and np.array_equal(Gs[1], Gu[1] * sc), name
        err = np.abs((Gs[0][I, J] - rh) + (Gs[1][I, J] - rl))
        assert np.all(err <= tol), (name, float(np.max(err / AB)))
        del Gu, Gs
