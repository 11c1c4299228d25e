"""GPU checks of dd_gemm_noalloc, the entry point that allocates nothing.

Its workspace is the library's fixed scratch array, and it launches the same
kernels as dd_gemm_ex, so every result must equal dd_gemm_ex's bit for bit.
The scratch array keeps the previous call's contents: two calls in a row,
the second smaller, check that nothing of the first leaks into the second.
"""
import numpy as np
import pytest

from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import make_problem
from tests.gpuhelp import down, log, up

pytestmark = pytest.mark.gpu


def _shape(P, transa, transb):
    A, B = P["A"][0], P["B"][0]
    m = A.shape[1] if transa else A.shape[0]
    k = A.shape[0] if transa else A.shape[1]
    n = B.shape[0] if transb else B.shape[1]
    return m, n, k


def _both(P, *, transa=False, transb=False, opts=None, flags=False):
    """The problem through dd_gemm_ex (library workspace) and dd_gemm_noalloc;
    returns both results (and both flag bitmaps when asked for)."""
    import torch
    m, n, k = _shape(P, transa, transb)
    A = (up(P["A"][0]), up(P["A"][1]))
    B = (up(P["B"][0]), up(P["B"][1]))
    lda, ldb, ldc = max(1, P["A"][0].shape[0]), max(1, P["B"][0].shape[0]), max(1, m)
    outs = []
    for fn in ("ex", "noalloc"):
        Ch, Cl = up(P["C"][0]), up(P["C"][1])
        o = dict(opts or {})
        fl = None
        if flags:
            fl = torch.full(((m * n + 31) // 32,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
            o["flags_out"] = fl.data_ptr()
        if fn == "ex":
            st = dg.dd_gemm_ex(int(transa), int(transb), m, n, k, A[0], A[1], lda, B[0], B[1], ldb,
                               Ch, Cl, ldc, opts=o)
        else:
            st = dg.dd_gemm_noalloc(int(transa), int(transb), m, n, k, A[0], A[1], lda, B[0], B[1], ldb,
                                    Ch, Cl, ldc, opts=o)
        dg.check(st, "dd_gemm_" + fn)
        torch.cuda.synchronize()
        outs.append(((down(Ch), down(Cl)), None if fl is None else fl.cpu().numpy()))
    return outs


def _same(a, b):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("opts", [
    None,
    {"kc": 128},
    {"scaling": dg.DD_SCALING_PANEL | dg.DD_SCALING_BALANCE},
    {"algo": dg.DD_ALGO_SLICES_BF16},
    {"algo": dg.DD_ALGO_SLICES_I8},
])
def test_two_calls_in_a_row_second_smaller(opts):
    variant = "panels" if opts and opts.get("scaling") else "scaled"
    for (m, n, k) in [(700, 520, 900), (130, 70, 257)]:
        log("noalloc opts=%s shape=%dx%dx%d" % (opts, m, n, k))
        P = make_problem(m, n, k, cfg=40, variant=variant)
        (ref, _), (got, _) = _both(P, opts=opts)
        _same(got, ref)


def test_transposes_and_flags():
    for (m, n, k) in [(300, 200, 600), (33, 17, 40)]:
        log("noalloc transposed + flags shape=%dx%dx%d" % (m, n, k))
        P = make_problem(m, n, k, cfg=41)
        P["A"] = (np.asfortranarray(P["A"][0].T), np.asfortranarray(P["A"][1].T))
        P["B"] = (np.asfortranarray(P["B"][0].T), np.asfortranarray(P["B"][1].T))
        (ref, fref), (got, fgot) = _both(P, transa=True, transb=True, flags=True)
        _same(got, ref)
        assert np.array_equal(fgot, fref)


def test_rejects_problems_beyond_the_scratch_and_leaves_c_alone():
    import torch
    m = n = k = 1408   # the cascade needs about 172 MiB, above the 128 MiB array
    assert dg.dd_gemm_workspace_size(0, 0, m, n, k) > dg.DD_NOALLOC_SCRATCH_BYTES
    log("noalloc oversize %d^3" % m)
    A = torch.zeros((k, m), dtype=torch.float64, device="cuda")
    B = torch.zeros((n, k), dtype=torch.float64, device="cuda")
    Ch = torch.full((n, m), 1.5, dtype=torch.float64, device="cuda")
    Cl = torch.full((n, m), 2.0 ** -60, dtype=torch.float64, device="cuda")
    st = dg.dd_gemm_noalloc(0, 0, m, n, k, A, A, m, B, B, k, Ch, Cl, m)
    assert st == dg.DD_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((Ch == 1.5).all()) and bool((Cl == 2.0 ** -60).all())
    # the unfused form (vendor BLAS) is refused as an option
    st = dg.dd_gemm_noalloc(0, 0, 8, 8, 8, A, A, m, B, B, k, Ch, Cl, m,
                            opts={"algo": dg.DD_ALGO_SIMPLE_UNFUSED})
    assert st == -15
    # a problem that fits right after the refusal still runs
    P = make_problem(64, 64, 64, cfg=42)
    (ref, _), (got, _) = _both(P)
    _same(got, ref)
