"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects invalid arguments on the host before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2303_04353_amd import ddgemm as dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddgemm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:dd|td)_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert set(declared_symbols()) == set(dg.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(dg.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    assert dg.dd_version() >= 100
    assert "success" in dg.dd_status_string(0)
    assert "gfx950" in dg.dd_status_string(dg.DD_ERR_UNSUPPORTED)
    assert "invalid" in dg.dd_status_string(-4)


@pytest.mark.parametrize("args,want", [
    ((-1, 2, 3, 0, 0, 1, 0, 0, 3, 0, 0, 1), -1),
    ((2, -1, 3, 0, 0, 2, 0, 0, 3, 0, 0, 2), -2),
    ((2, 2, -3, 0, 0, 2, 0, 0, 1, 0, 0, 2), -3),
    ((4, 4, 4, 8, 8, 3, 16, 16, 4, 32, 40, 4), -6),     # lda < m
    ((4, 4, 4, 8, 8, 4, 16, 16, 3, 32, 40, 4), -9),     # ldb < k
    ((4, 4, 4, 8, 8, 4, 16, 16, 4, 32, 40, 3), -12),    # ldc < m
    ((4, 4, 4, 0, 8, 4, 16, 16, 4, 1 << 30, 1 << 31, 4), -4),     # A_hi NULL
    ((4, 4, 4, 8, 8, 4, 16, 16, 4, 0, 1 << 31, 4), -10),          # C_hi NULL
    ((4, 4, 4, 8, 16, 4, 1 << 20, 1 << 21, 4, 8, 1 << 22, 4), -10),  # C_hi overlaps A_hi
    ((4, 4, 4, 8, 16, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 22, 4), -11),  # C_lo overlaps C_hi
    ((4, 4, 4, 8, 16, 1 << 61, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4), -6),   # A's extent overflows
    ((4, 4, 4, 8, 16, 4, 1 << 20, 1 << 21, 1 << 61, 1 << 22, 1 << 23, 4), -9),   # B's extent overflows
    ((4, 4, 4, 8, 16, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 1 << 61), -12),  # C's extent overflows
])
def test_invalid_arguments_rejected_on_host(args, want):
    assert dg.dd_gemm(*args, stream=0) == want


def test_ex_rejects_bad_ops_and_options():
    base = (4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 4)
    assert dg.dd_gemm_ex(2, 0, *base, stream=0) == -1
    assert dg.dd_gemm_ex(0, 7, *base, stream=0) == -2
    assert dg.dd_gemm_ex(0, 0, *base, opts={"kc": 6}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts={"algo": 9}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts={"tile": 7}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, workspace=None, ws_bytes=64, stream=0) == -15


def test_without_a_gpu_valid_calls_fail_cleanly():
    # No device in this container: a valid call must return an error status,
    # never crash or compute on the host.
    base = (4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 4)
    st = dg.dd_gemm(*base, stream=0)
    if st != dg.DD_OK:
        assert st in (dg.DD_ERR_HIP, dg.DD_ERR_UNSUPPORTED)


def test_workspace_size_formula():
    ws = dg.dd_gemm_workspace_size(0, 0, 100, 70, 300)
    mpad, npad, kpad = 128, 128, 304
    # packed planes: per 16-row (16-column) block 4 (7) planes over kpad, plus 544 doubles of padding
    need = 8 * (mpad + npad) + 8 * (mpad // 16) * (4 * 16 * kpad + 544) + 8 * (npad // 16) * (7 * 16 * kpad + 544)
    assert need <= ws <= need + 4 * 256
    assert dg.dd_gemm_workspace_size(0, 0, 100, 70, 300, {"algo": dg.DD_ALGO_DD_VALU}) == 0
    assert dg.dd_gemm_workspace_size(3, 0, 100, 70, 300) == 0
    assert dg.dd_gemm_workspace_size(0, 0, 0, 70, 300) == 0


def test_panel_scaling_option_and_workspace():
    m, n, k = 100, 70, 1000
    mpad, npad, kpad = 128, 128, 1008
    g = dg.dd_gemm_workspace_size(0, 0, m, n, k)
    # four rank-256 panels: three more sets of maxima and four sets of int32 exponents
    p = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"scaling": dg.DD_SCALING_PANEL})
    extra = 8 * 3 * (mpad + npad) + 4 * 4 * (mpad + npad)
    assert g + extra - 4 * 256 <= p <= g + extra + 4 * 256
    assert 8 * (mpad + npad) + 8 * 9 * 128 * kpad <= g
    # one panel: the global layout
    assert dg.dd_gemm_workspace_size(0, 0, m, n, 200, {"scaling": 1}) == dg.dd_gemm_workspace_size(0, 0, m, n, 200)
    # balancing: column / row maxima (8 B each) and an int32 exponent per padded inner index
    b = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"scaling": dg.DD_SCALING_BALANCE})
    assert g + 20 * 1008 <= b <= g + 20 * 1008 + 3 * 256
    pb = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"scaling": dg.DD_SCALING_PANEL | dg.DD_SCALING_BALANCE})
    assert pb == p + (b - g)
    for bad in ({"scaling": 4}, {"scaling": -1}, {"algo": dg.DD_ALGO_DD_VALU, "scaling": 1},
                {"algo": dg.DD_ALGO_SLICES_BF16, "scaling": 1}, {"algo": dg.DD_ALGO_SLICES_I8, "scaling": 2}):
        assert dg.dd_gemm_workspace_size(0, 0, m, n, k, bad) == 0, bad


def test_td_workspace_and_argument_checks():
    m, n, k = 100, 70, 300
    ws = dg.td_gemm_workspace_size(0, 0, m, n, k)
    mpad, npad, K4 = 128, 128, 304 // 4
    # maxima, then six packed digit planes per 16-row (16-column) block over
    # kpad, plus 544 doubles of padding per block
    need = 8 * (mpad + npad) + 8 * (mpad // 16 + npad // 16) * (6 * 64 * K4 + 544)
    assert need <= ws <= need + 4 * 256
    assert dg.td_gemm_workspace_size(0, 0, m, n, k, 64) == ws
    assert dg.td_gemm_workspace_size(0, 0, m, n, k, 6) == 0
    assert dg.td_gemm_workspace_size(2, 0, m, n, k) == 0 and dg.td_gemm_workspace_size(0, 0, 0, n, k) == 0
    p = 1 << 20
    base = dict(transa=0, transb=0, m=4, n=4, k=4, A0=p, A1=2 * p, A2=3 * p, lda=4, B0=4 * p, B1=5 * p, B2=6 * p,
                ldb=4, C0=7 * p, C1=8 * p, C2=9 * p, ldc=4)
    def call(**kw):
        a = dict(base, **kw)
        return dg.td_gemm_ex(a["transa"], a["transb"], a["m"], a["n"], a["k"], a["A0"], a["A1"], a["A2"], a["lda"],
                             a["B0"], a["B1"], a["B2"], a["ldb"], a["C0"], a["C1"], a["C2"], a["ldc"],
                             kc=a.get("kc", 0), stream=0)
    assert call(transa=3) == -1 and call(transb=3) == -2 and call(m=-1) == -3 and call(k=-2) == -5
    assert call(lda=3) == -9 and call(ldb=3) == -13 and call(ldc=3) == -17 and call(kc=10) == -20
    assert call(lda=1 << 61) == -9 and call(ldb=1 << 61) == -13 and call(ldc=1 << 61) == -17
    assert call(A1=0) == -7 and call(B2=0) == -12 and call(C0=0) == -14
    assert call(C1=7 * p + 8) == -15          # C planes overlap
    assert call(C2=2 * p) == -16              # C overlaps A
    assert call(m=0, C0=0) == dg.DD_OK         # nothing to do, nothing read


def test_simple_unfused_options_and_workspace():
    m, n, k = 100, 70, 300
    g = dg.dd_gemm_workspace_size(0, 0, m, n, k)
    u = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": dg.DD_ALGO_SIMPLE_UNFUSED})
    extra = 8 * (4 * m * k + 7 * k * n + 6 * m * n)
    assert g + extra <= u <= g + extra + 4 * 256
    assert dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": dg.DD_ALGO_SIMPLE_UNFUSED, "kc": 64}) == u
    for bad in ({"algo": dg.DD_ALGO_SIMPLE_UNFUSED, "scaling": 1}, {"algo": dg.DD_ALGO_SIMPLE_UNFUSED, "slices": 4},
                {"algo": dg.DD_ALGO_SIMPLE_UNFUSED, "kc": 6}):
        assert dg.dd_gemm_workspace_size(0, 0, m, n, k, bad) == 0, bad


def test_slices_options_and_workspace():
    bf, f16 = dg.DD_ALGO_SLICES_BF16, dg.DD_ALGO_SLICES_F16
    m, n, k = 100, 70, 300
    mpad, npad, kpad = 128, 128, 320
    # default BF16: 14 slices of 8 bits, plus the upper pass's groups 3 and 4
    ws = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": bf})
    pad = 4352 * (mpad // 32 + npad // 32)   # 4 KiB + 256 B after every 32-row (column) block
    need = 8 * (mpad + npad) + 2 * 14 * (mpad + npad) * kpad + pad + 8 * 2 * mpad * npad
    assert need <= ws <= need + 6 * 256
    # nine slices or fewer run in one pass: no group planes
    ws9 = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": bf, "slices": 9})
    need9 = 8 * (mpad + npad) + 2 * 9 * (mpad + npad) * kpad + pad
    assert need9 <= ws9 <= need9 + 6 * 256
    assert dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": f16}) > 0
    for bad in ({"algo": bf, "slice_bits": 10}, {"algo": bf, "slices": 17}, {"algo": f16, "slice_bits": 10},
                {"algo": bf, "kc": 256}, {"algo": 0, "slices": 4}, {"algo": 1, "slice_bits": 8},
                {"algo": f16, "slice_bits": 12, "slices": 1}, {"algo": 7}):
        assert dg.dd_gemm_workspace_size(0, 0, m, n, k, bad) == 0, bad
    assert dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": f16, "slice_bits": 11, "slices": 1}) > 0
    # INT8: 16 slices of 7 bits, one byte each, k padded to 128, groups 3..5 of the upper pass
    i8 = dg.DD_ALGO_SLICES_I8
    ws8 = dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": i8})
    need8 = 8 * (mpad + npad) + 16 * (mpad + npad) * 384 + 4352 * (mpad // 32 + npad // 32) + 8 * 3 * mpad * npad
    assert need8 <= ws8 <= need8 + 6 * 256
    assert dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": i8, "slice_bits": 8}) == 0
    assert dg.dd_gemm_workspace_size(0, 0, m, n, k, {"algo": 7}) == 0
    base = (4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 4)
    assert dg.dd_gemm_ex(0, 0, *base, opts={"algo": bf, "slices": 20}, stream=0) == -17


def test_slices_split_rejects_bad_arguments():
    assert dg.dd_slices_split(2, 0, 4, 4, 8, 16, 4, 0, 0, 0, 32, 64, stream=0) == -1
    assert dg.dd_slices_split(0, 2, 4, 4, 8, 16, 4, 0, 0, 0, 32, 64, stream=0) == -2
    assert dg.dd_slices_split(0, 0, -4, 4, 8, 16, 4, 0, 0, 0, 32, 64, stream=0) == -3
    assert dg.dd_slices_split(0, 0, 4, 4, 8, 16, 3, 0, 0, 0, 32, 64, stream=0) == -7
    assert dg.dd_slices_split(0, 0, 4, 4, 8, 16, 4, 3, 0, 0, 32, 64, stream=0) == -8
    assert dg.dd_slices_split(0, 0, 4, 4, 8, 16, 4, 2, 0, 8, 32, 64, stream=0) == -9   # w = 8 overflows int8
    assert dg.dd_slices_split(0, 0, 4, 4, 8, 16, 4, 0, 0, 10, 32, 64, stream=0) == -9
    assert dg.dd_slices_split(0, 0, 4, 4, 0, 16, 4, 0, 0, 0, 32, 64, stream=0) == -5
    assert dg.dd_slices_split(0, 0, 4, 4, 8, 16, 4, 0, 0, 0, 0, 64, stream=0) == -11


def test_noalloc_rejects_bad_arguments_on_host():
    base = (4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 4)
    assert dg.dd_gemm_noalloc(2, 0, *base, stream=0) == -1
    assert dg.dd_gemm_noalloc(0, 0, 4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 3,
                              stream=0) == -14
    assert dg.dd_gemm_noalloc(0, 0, *base, opts={"kc": 6}, stream=0) == -15
    # the unfused form runs the vendor BLAS, which may allocate
    assert dg.dd_gemm_noalloc(0, 0, *base, opts={"algo": dg.DD_ALGO_SIMPLE_UNFUSED}, stream=0) == -15
    assert dg.DD_NOALLOC_SCRATCH_BYTES == 128 << 20
    # the largest square cascade the scratch array holds, and the first one it does not
    assert dg.dd_gemm_workspace_size(0, 0, 1216, 1216, 1216) <= dg.DD_NOALLOC_SCRATCH_BYTES
    assert dg.dd_gemm_workspace_size(0, 0, 1217, 1217, 1217) > dg.DD_NOALLOC_SCRATCH_BYTES


def test_vector_calls_reject_bad_arguments_on_host():
    # dd_scal(n, alpha, x_hi, x_lo, incx, y_hi, y_lo, incy): alpha is a device pointer
    assert dg.dd_scal(-1, 8, 16, 24, 1, 32, 40, 1, stream=0) == -1
    assert dg.dd_scal(4, 0, 16, 24, 1, 1 << 20, 1 << 21, 1, stream=0) == -2
    assert dg.dd_scal(4, 8, 1 << 20, 1 << 21, 0, 1 << 22, 1 << 23, 1, stream=0) == -5
    assert dg.dd_scal(4, 8, 1 << 20, 1 << 21, 1, 1 << 20, 1 << 23, 1, stream=0) == -6   # y_hi over x_hi, not equal pair
    assert dg.dd_scal(4, 8, 1 << 20, 1 << 21, 1, 1 << 22, 1 << 22, 1, stream=0) == -7  # y_lo over y_hi
    # dd_add(n, x_hi, x_lo, incx, y_hi, y_lo, incy, z_hi, z_lo, incz)
    x = (1 << 20, 1 << 21)
    y = (1 << 22, 1 << 23)
    assert dg.dd_add(-1, *x, 1, *y, 1, 1 << 24, 1 << 25, 1, stream=0) == -1
    assert dg.dd_add(4, 0, x[1], 1, *y, 1, 1 << 24, 1 << 25, 1, stream=0) == -2
    assert dg.dd_add(4, *x, 1, *y, 0, 1 << 24, 1 << 25, 1, stream=0) == -7
    assert dg.dd_add(4, *x, 1, *y, 1, 1 << 24, 1 << 25, 0, stream=0) == -10
    assert dg.dd_add(4, *x, 1, *y, 1, x[0] + 8, 1 << 25, 1, stream=0) == -8          # z_hi inside x_hi
    assert dg.dd_add(4, *x, 1, *y, 1, 1 << 24, y[1] + 16, 1, stream=0) == -9         # z_lo inside y_lo
    assert dg.dd_add(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, stream=0) == 0


def test_tile_and_tuner_options_checked_on_host():
    base = (4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 4)
    assert dg.dd_gemm_ex(0, 0, *base, opts={"tile": 4}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts={"tile": -1}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts={"tile": 2, "algo": dg.DD_ALGO_DD_VALU}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts={"use_tuned": 2}, stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts={"use_tuned": 1, "algo": dg.DD_ALGO_SLICES_BF16}, stream=0) == -17
    assert dg.dd_gemm_workspace_size(0, 0, 100, 70, 300, {"tile": 2}) == dg.dd_gemm_workspace_size(0, 0, 100, 70, 300)
    assert dg.dd_tune([4], [4], [4], repeats=0, stream=0)[0] == -6
    assert dg.dd_tune([4], [4], [4], opts={"algo": dg.DD_ALGO_SLICES_BF16}, stream=0)[0] == -5
    assert dg.dd_tune([4], [4], [4], opts={"tile": 1}, stream=0)[0] == -5
    assert dg.dd_tune([4], [-4], [4], stream=0)[0] == -2
    assert dg.dd_tune([], [], [], stream=0)[0] in (0, dg.DD_ERR_HIP, dg.DD_ERR_UNSUPPORTED)


def test_on_load_options_and_workspace():
    base = (4, 4, 4, 1 << 20, 1 << 21, 4, 1 << 22, 1 << 23, 4, 1 << 24, 1 << 25, 4)
    o = {"algo": dg.DD_ALGO_CASCADE_ON_LOAD}
    assert dg.dd_gemm_ex(0, 0, *base, opts=dict(o, scaling=dg.DD_SCALING_PANEL), stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts=dict(o, tile=dg.DD_TILE_32x64), stream=0) == -17
    assert dg.dd_gemm_ex(0, 0, *base, opts=dict(o, use_tuned=1), stream=0) == -17
    # only the row and column maxima: 8 (mpad + npad) bytes, 256-byte aligned pieces
    assert dg.dd_gemm_workspace_size(0, 0, 100, 70, 300, o) == 8 * 128 + 8 * 128
    assert dg.dd_gemm_workspace_size(0, 0, 100, 70, 300, dict(o, tile=dg.DD_TILE_64x64)) == 8 * 256


def test_one_shot_batched_checks_on_host_and_workspace_size():
    m, n, k = [64, 100], [32, 70], [16, 300]
    ld = [128, 128]
    ptrs = (1 << 20, 1 << 21, ld, 1 << 22, 1 << 23, ld, 1 << 24, 1 << 25, ld)
    assert dg.dd_gemm_batched(-1, m, n, k, *ptrs, stream=0) == -1
    assert dg.dd_gemm_batched(2, m, n, k, *ptrs, workspace=None, ws_bytes=4096, stream=0) == -15
    assert dg.dd_gemm_batched(2, m, n, k, *ptrs, workspace=(1 << 26) + 8, ws_bytes=1 << 30, stream=0) == -14
    assert dg.dd_gemm_batched(2, m, n, k, *ptrs, opts={"kc": 6}, stream=0) == -16
    assert dg.dd_gemm_batched(2, m, n, k, *ptrs, opts={"scaling": dg.DD_SCALING_PANEL}, stream=0) == -16
    assert dg.dd_gemm_batched(2, [64, -1], n, k, *ptrs, stream=0) == -2
    assert dg.dd_gemm_batched(2, m, n, k, 1 << 20, 1 << 21, [63, 128], 1 << 22, 1 << 23, ld, 1 << 24, 1 << 25, ld,
                              stream=0) == -7
    # workspace: a 256-byte counter, the exponent words of both problems
    # (rows and columns rounded up to 64), then the packed planes: per
    # 16-row block of A the single GEMM's 4 planes, per 16-column block of B
    # 5 (the single GEMM stores 7), over k rounded up to 16, plus 544
    # doubles of padding per block
    ws = dg.dd_gemm_batched_workspace_size(2, m, n, k)
    exps = 8 * (64 + 64 + 128 + 128)
    planes = 0
    for mi, ni, ki in zip(m, n, k):
        mp, np_, kp = -(-mi // 64) * 64, -(-ni // 64) * 64, -(-ki // 16) * 16
        planes += 8 * (mp // 16) * (4 * 16 * kp + 544) + 8 * (np_ // 16) * (5 * 16 * kp + 544)
        single = dg.dd_gemm_workspace_size(0, 0, mi, ni, ki)
        assert single - 8 * (mp + np_) == 8 * (mp // 16) * (4 * 16 * kp + 544) + 8 * (np_ // 16) * (7 * 16 * kp + 544)
    assert ws >= 256 + exps + planes - 2 * 256 and ws <= 256 + exps + planes + 4 * 256
    assert dg.dd_gemm_batched_workspace_size(2, m, n, [16, 600]) > ws
    assert dg.dd_gemm_batched_workspace_size(2, m, n, k, opts={"kc": 6}) == 0
    assert dg.dd_gemm_batched_workspace_size(-1, m, n, k) == 0
    # problems with a zero dimension take no room
    assert dg.dd_gemm_batched_workspace_size(3, m + [500], n + [0], k + [500]) == ws
