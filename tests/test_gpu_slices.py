"""GPU parity of the narrow-slice variant (BF16/FP16 slices, C ABI) against
the oracle.

Every level sum is an exact integer and the split and the FP64x2 combine are
fixed sequences of round-to-nearest operations, so the device result must
equal the oracle's bit for bit (hi and lo words):

* slices and exponents of dd_slices_split against the oracle's split;
* C := op(A) op(B) + C for ragged shapes, both formats, several (w, s),
  uniform and ill-scaled inputs, transposed storage, a chunked inner
  dimension, and sampled entries of the 4096^3 workload;
* accuracy against the FP64x2 oracle within 64 k 2^-104 (|A||B|)_ij;
* edge cases: k = 0, empty, non-finite rows and columns.
"""
import numpy as np
import pytest

from oracle import slices as sl
from oracle.ref import dd_gemm_ref, dd_gemm_ref_entries
from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import make_problem, sample_entries
from tests.gpuhelp import dd_diff, log, fp64x2_tolerance, run_gemm, up

pytestmark = pytest.mark.gpu

BF, F16, I8 = dg.DD_ALGO_SLICES_BF16, dg.DD_ALGO_SLICES_F16, dg.DD_ALGO_SLICES_I8
FMT = {BF: "bf16", F16: "f16", I8: "i8"}


def _bits(a, fmt):
    """16-bit form of integer-valued float64 slices: the BF16 (0) or FP16 (1)
    pattern, or the INT8 value sign-extended (2)."""
    if fmt == 1:
        return a.astype(np.float16).view(np.uint16)
    if fmt == 2:
        return a.astype(np.int16).view(np.uint16)
    return (a.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("shape", [(37, 50), (64, 256), (129, 300), (1, 1), (70, 33)])
@pytest.mark.parametrize("variant", ["uniform", "scaled"])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("f16,w,s", [(0, 8, 14), (1, 9, 12), (0, 9, 16), (1, 11, 1), (2, 7, 16), (2, 5, 3)])
def test_split_bitwise(shape, variant, trans, f16, w, s):
    import torch
    rows, cols = shape
    log(f"slices split shape={shape} variant={variant} trans={trans} f16={f16} w={w} s={s}")
    P = make_problem(rows, cols, cols, cfg=40, variant=variant)
    X = P["A"]
    stored = (np.asfortranarray(X[0].T), np.asfortranarray(X[1].T)) if trans else X
    for side in (0, 1):
        nexp = rows if side == 0 else cols
        exps = torch.zeros(max(nexp, 1), dtype=torch.int32, device="cuda")
        out = torch.zeros(s * rows * cols, dtype=torch.int16, device="cuda")
        st = dg.dd_slices_split(side, int(trans), rows, cols, up(stored[0]), up(stored[1]),
                                max(1, stored[0].shape[0]), f16, s, w, exps, out)
        dg.check(st, "dd_slices_split")
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint16).reshape(s, cols, rows)
        axis = 1 if side == 0 else 0
        e = sl.slice_exponents(X[0], X[1], axis=axis)
        want, _ = sl.split_slices(X[0], X[1], e, axis, w, s)
        assert np.array_equal(exps.cpu().numpy()[:nexp], e)
        for t in range(s):
            assert np.array_equal(got[t].T, _bits(want[t], f16)), (side, t)


CASES = [((37, 50, 300), "uniform"), ((130, 70, 1000), "scaled"), ((1, 1, 1), "uniform"),
         ((64, 64, 64), "scaled"), ((65, 65, 65), "uniform"), ((200, 128, 520), "uniform"),
         ((3, 200, 17), "scaled"), ((128, 3, 257), "uniform")]


@pytest.mark.parametrize("shape,variant", CASES)
@pytest.mark.parametrize("algo,w,s", [(BF, 8, 14), (BF, 9, 12), (F16, 9, 12), (BF, 7, 16), (BF, 8, 9),
                                      (BF, 6, 4), (F16, 11, 1), (I8, 7, 16), (I8, 7, 12), (I8, 6, 9), (I8, 4, 2)])
def test_gemm_bitwise_against_oracle(shape, variant, algo, w, s):
    m, n, k = shape
    log(f"slices gemm {shape} {variant} algo={algo} w={w} s={s}")
    P = make_problem(m, n, k, cfg=41, variant=variant)
    got = run_gemm(P["A"], P["B"], P["C"], algo=algo, slices=s, slice_bits=w)
    want = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, fmt=FMT[algo])
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_int8_equals_bf16_at_the_same_widths():
    m, n, k = 150, 90, 700
    P = make_problem(m, n, k, cfg=48, variant="scaled")
    a = run_gemm(P["A"], P["B"], P["C"], algo=I8, slices=16, slice_bits=7)
    b = run_gemm(P["A"], P["B"], P["C"], algo=BF, slices=16, slice_bits=7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("variant", ["uniform", "scaled"])
@pytest.mark.parametrize("algo", [BF, F16, I8])
def test_defaults_meet_the_fp64x2_tolerance(variant, algo):
    m, n, k = 150, 120, 700
    log(f"slices default accuracy algo={algo} {variant}")
    P = make_problem(m, n, k, cfg=42, variant=variant)
    got = run_gemm(P["A"], P["B"], P["C"], algo=algo)
    ref = dd_gemm_ref(P["A"], P["B"], P["C"])[:2]
    assert np.all(dd_diff(got, ref) <= fp64x2_tolerance(P["A"], P["B"], k))
    w, s = (7, 16) if algo == I8 else (8, 14)
    want = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, fmt=FMT[algo])
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("ta,tb", [(True, False), (False, True), (True, True)])
def test_transposes_are_bit_identical(ta, tb):
    m, n, k = 70, 90, 130
    P = make_problem(m, n, k, cfg=43, variant="scaled")
    base = run_gemm(P["A"], P["B"], P["C"], algo=BF)
    A = (np.asfortranarray(P["A"][0].T), np.asfortranarray(P["A"][1].T)) if ta else P["A"]
    B = (np.asfortranarray(P["B"][0].T), np.asfortranarray(P["B"][1].T)) if tb else P["B"]
    got = run_gemm(A, B, P["C"], transa=ta, transb=tb, algo=BF)
    assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])


@pytest.mark.parametrize("algo,w,s", [(BF, 9, 12), (I8, 7, 16)])
def test_chunked_inner_dimension(algo, w, s):
    k = sl.chunk_limit(w, s, FMT[algo]) + 40
    log(f"slices chunked algo={algo} k={k}")
    P = make_problem(5, 66, k, cfg=44)
    got = run_gemm(P["A"], P["B"], P["C"], algo=algo, slices=s, slice_bits=w)
    want = sl.slices_gemm(P["A"], P["B"], P["C"], w=w, s=s, fmt=FMT[algo])
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_zero_inner_dimension_and_empty():
    P = make_problem(5, 6, 0, cfg=45)
    got = run_gemm(P["A"], P["B"], P["C"], algo=BF)
    assert np.array_equal(got[0], P["C"][0]) and np.array_equal(got[1], P["C"][1])
    st = dg.dd_gemm_ex(0, 0, 0, 5, 3, None, None, 1, None, None, 3, None, None, 1, opts={"algo": BF})
    assert st == dg.DD_OK


@pytest.mark.parametrize("algo", [BF, I8])
def test_non_finite_rows_and_columns_give_nan(algo):
    P = make_problem(40, 30, 50, cfg=46)
    A = (P["A"][0].copy(), P["A"][1].copy())
    B = (P["B"][0].copy(), P["B"][1].copy())
    A[0][7, 3] = np.inf
    B[0][11, 4] = np.nan
    got = run_gemm(A, B, P["C"], algo=algo)
    assert np.all(np.isnan(got[0][7, :])) and np.all(np.isnan(got[0][:, 4]))
    ok = np.ones_like(got[0], dtype=bool)
    ok[7, :] = False
    ok[:, 4] = False
    w, s = (7, 16) if algo == I8 else (8, 14)
    want = sl.slices_gemm(A, B, P["C"], w=w, s=s, fmt=FMT[algo])
    assert np.array_equal(got[0][ok], want[0][ok]) and np.array_equal(got[1][ok], want[1][ok])


def test_caller_workspace_equals_internal():
    import torch
    m, n, k = 100, 80, 200
    P = make_problem(m, n, k, cfg=47)
    base = run_gemm(P["A"], P["B"], P["C"], algo=BF)
    opts = {"algo": BF}
    nbytes = dg.dd_gemm_workspace_size(0, 0, m, n, k, opts)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    Ch, Cl = up(P["C"][0]), up(P["C"][1])
    st = dg.dd_gemm_ex(0, 0, m, n, k, up(P["A"][0]), up(P["A"][1]), m, up(P["B"][0]), up(P["B"][1]), k,
                       Ch, Cl, m, workspace=ws, ws_bytes=nbytes, opts=opts)
    dg.check(st)
    torch.cuda.synchronize()
    assert np.array_equal(dg.colmajor_from_device(Ch), base[0])
    assert np.array_equal(dg.colmajor_from_device(Cl), base[1])
    assert dg.dd_gemm_ex(0, 0, m, n, k, up(P["A"][0]), up(P["A"][1]), m, up(P["B"][0]), up(P["B"][1]), k,
                         Ch, Cl, m, workspace=ws, ws_bytes=nbytes - 1, opts=opts) == dg.DD_ERR_WORKSPACE


@pytest.mark.parametrize("algo", [BF, I8])
@pytest.mark.parametrize("variant", ["uniform", "scaled"])
def test_full_size_sampled_parity_4096(variant, algo):
    import torch
    n = 4096
    log(f"slices 4096^3 {variant}: generating")
    P = make_problem(n, n, n, cfg=2, variant=variant)
    Ah, Al, Bh, Bl = (up(x) for x in (*P["A"], *P["B"]))
    Ch, Cl = up(P["C"][0]), up(P["C"][1])
    log("slices 4096^3: running")
    dg.check(dg.dd_gemm_ex(0, 0, n, n, n, Ah, Al, n, Bh, Bl, n, Ch, Cl, n, opts={"algo": algo}))
    torch.cuda.synchronize()
    I, J = sample_entries(n, n, 48, seed=11)
    gh = Ch.T.cpu().numpy()[I, J]
    gl = Cl.T.cpu().numpy()[I, J]
    log("slices 4096^3: oracle entries")
    w, s = (7, 16) if algo == I8 else (8, 14)
    wh, wl = sl.slices_gemm_entries(P["A"], P["B"], P["C"], I, J, w=w, s=s, fmt=FMT[algo])
    assert np.array_equal(gh, wh) and np.array_equal(gl, wl)
    rh, rl, _ = dd_gemm_ref_entries(P["A"], P["B"], P["C"], I, J)
    AB = np.array([np.abs(P["A"][0][i]) @ np.abs(P["B"][0][:, j]) for i, j in zip(I, J)])
    assert np.all(np.abs((gh - rh) + (gl - rl)) <= 64 * n * 2.0 ** -104 * AB)
