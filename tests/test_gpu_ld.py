"""GPU checks of leading dimensions larger than the stored row count.

Each operand is embedded in a larger column-major buffer (lda = rows + 3,
ldb = rows + 5, ldc = m + 7); the padding rows of A and B hold NaN, so a
kernel that reads them turns results into NaN, and the padding rows of C
hold a sentinel that must survive the call.  Every path must give the same
bits as with tight leading dimensions (the packed planes, the slices and
the per-entry arithmetic do not depend on ld), and that result is checked
against the FP64x2 oracle within the tolerance.
"""
import numpy as np
import pytest

from oracle.ref import dd_gemm_ref
from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import make_problem
from tests.gpuhelp import dd_diff, log, fp64x2_tolerance, run_gemm

pytestmark = pytest.mark.gpu

SENTINEL = 12345.678


def _padded(X, pad, fill):
    """Device buffer of shape (cols, rows + pad) holding X (rows x cols,
    column-major) in its first rows; the rest is `fill`."""
    import torch
    rows, cols = X.shape
    t = torch.full((cols, rows + pad), fill, dtype=torch.float64)
    t[:, :rows] = torch.from_numpy(np.ascontiguousarray(X.T))
    return t.cuda()


def run_padded(P, *, transa=False, transb=False, opts=None, pads=(3, 5, 7), noalloc=False):
    import torch
    A, B, C = P["A"], P["B"], P["C"]
    m = A[0].shape[1] if transa else A[0].shape[0]
    k = A[0].shape[0] if transa else A[0].shape[1]
    n = B[0].shape[0] if transb else B[0].shape[1]
    pa, pb, pc = pads
    Ah, Al = _padded(A[0], pa, np.nan), _padded(A[1], pa, np.nan)
    Bh, Bl = _padded(B[0], pb, np.nan), _padded(B[1], pb, np.nan)
    Ch, Cl = _padded(C[0], pc, SENTINEL), _padded(C[1], pc, -SENTINEL)
    lda, ldb, ldc = A[0].shape[0] + pa, B[0].shape[0] + pb, m + pc
    st = dg.dd_gemm_ex(int(transa), int(transb), m, n, k, Ah, Al, lda, Bh, Bl, ldb, Ch, Cl, ldc, opts=opts)
    dg.check(st, "dd_gemm_ex")
    torch.cuda.synchronize()
    ch, cl = Ch.cpu().numpy(), Cl.cpu().numpy()
    assert np.all(ch[:, m:] == SENTINEL) and np.all(cl[:, m:] == -SENTINEL), "padding of C changed"
    return np.asfortranarray(ch[:, :m].T), np.asfortranarray(cl[:, :m].T)


def _t(X):
    return (np.asfortranarray(X[0].T), np.asfortranarray(X[1].T))


CASES = [
    ("cascade", {}),
    ("cascade kc=64", {"kc": 64}),
    ("cascade panel", {"scaling": dg.DD_SCALING_PANEL, "kc": 128}),
    ("cascade balance", {"scaling": dg.DD_SCALING_BALANCE}),
    ("cascade panel+balance", {"scaling": dg.DD_SCALING_PANEL | dg.DD_SCALING_BALANCE, "kc": 128}),
    ("dd_valu", {"algo": dg.DD_ALGO_DD_VALU}),
    ("slices bf16", {"algo": dg.DD_ALGO_SLICES_BF16}),
    ("slices f16", {"algo": dg.DD_ALGO_SLICES_F16}),
    ("slices i8", {"algo": dg.DD_ALGO_SLICES_I8}),
    ("unfused", {"algo": dg.DD_ALGO_SIMPLE_UNFUSED, "kc": 128}),
]


@pytest.mark.parametrize("name,opts", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_padded_leading_dimensions_bitwise(name, opts, ta, tb):
    m, n, k = 133, 70, 300
    log(f"ld padded: {name} transa={ta} transb={tb} shape={m}x{n}x{k}")
    P = make_problem(m, n, k, cfg=50, variant="scaled")
    Q = dict(P)
    if ta:
        Q["A"] = _t(P["A"])
    if tb:
        Q["B"] = _t(P["B"])
    kw = {key: v for key, v in opts.items()}
    tight = run_gemm(Q["A"], Q["B"], Q["C"], transa=ta, transb=tb, algo=kw.pop("algo", dg.DD_ALGO_CASCADE_F64),
                     kc=kw.pop("kc", 0), scaling=kw.pop("scaling", 0))
    got = run_padded(Q, transa=ta, transb=tb, opts=opts)
    assert np.array_equal(got[0], tight[0]) and np.array_equal(got[1], tight[1])
    if not (ta or tb):
        R = dd_gemm_ref(P["A"], P["B"], P["C"])[:2]
        assert np.all(dd_diff(got, R) <= fp64x2_tolerance(P["A"], P["B"], k))


def test_padded_batched_plan_bitwise():
    """A batched plan with lda > m, ldb > k, ldc > m for every problem: each
    result equals the single call with tight leading dimensions."""
    import torch
    shapes = [(37, 50, 300), (64, 64, 64), (130, 70, 1000), (17, 200, 33), (1, 1, 1), (65, 3, 257)]
    pads = [(3, 5, 7), (1, 1, 1), (64, 2, 9), (5, 128, 3), (2, 3, 4), (11, 7, 1)]
    P = [make_problem(m, n, k, cfg=51, salt=i) for i, (m, n, k) in enumerate(shapes)]
    A = [(_padded(p["A"][0], pa, np.nan), _padded(p["A"][1], pa, np.nan)) for p, (pa, _, _) in zip(P, pads)]
    B = [(_padded(p["B"][0], pb, np.nan), _padded(p["B"][1], pb, np.nan)) for p, (_, pb, _) in zip(P, pads)]
    C = [(_padded(p["C"][0], pc, SENTINEL), _padded(p["C"][1], pc, -SENTINEL)) for p, (_, _, pc) in zip(P, pads)]
    ptrs = lambda lst, w: torch.tensor([t[w].data_ptr() for t in lst], dtype=torch.int64, device="cuda")
    ms, ns, ks = [s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes]
    lda = [m + p[0] for m, p in zip(ms, pads)]
    ldb = [k + p[1] for k, p in zip(ks, pads)]
    ldc = [m + p[2] for m, p in zip(ms, pads)]
    log("ld padded: batched plan of %d problems" % len(shapes))
    st, plan = dg.dd_batched_plan_create(len(shapes), ms, ns, ks, lda, ldb, ldc)
    dg.check(st, "dd_batched_plan_create")
    try:
        dg.check(dg.dd_gemm_batched_exec(plan, ptrs(A, 0), ptrs(A, 1), ptrs(B, 0), ptrs(B, 1),
                                         ptrs(C, 0), ptrs(C, 1)), "dd_gemm_batched_exec")
        torch.cuda.synchronize()
    finally:
        dg.dd_batched_plan_destroy(plan)
    for i, (m, n, k) in enumerate(shapes):
        ch, cl = C[i][0].cpu().numpy(), C[i][1].cpu().numpy()
        assert np.all(ch[:, m:] == SENTINEL) and np.all(cl[:, m:] == -SENTINEL), i
        want = run_gemm(P[i]["A"], P[i]["B"], P[i]["C"])
        assert np.array_equal(ch[:, :m].T, want[0]) and np.array_equal(cl[:, :m].T, want[1]), i
