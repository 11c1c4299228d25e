"""ctypes binding of ``libddgemm.so``: the C ABI of include/ddgemm.h, same names.

Only argument marshalling happens here: device pointers are taken from torch
tensors (``.data_ptr()``) or passed as integers, the stream defaults to
torch's current stream.  Every step of the computation runs in the HIP
library; if it is not built, :func:`lib` raises.

Matrices are column-major as in BLAS.  A column-major ``rows x cols`` matrix
is held in a contiguous torch tensor of shape ``(cols, rows)`` (its
transpose), see :func:`colmajor_to_device` / :func:`colmajor_from_device`.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddgemm.so")

DD_OK = 0
DD_ERR_HIP = 1
DD_ERR_WORKSPACE = 2
DD_ERR_UNSUPPORTED = 3
DD_ERR_INTERNAL = 4
DD_OP_N = 0
DD_OP_T = 1
DD_ALGO_CASCADE_F64 = 0
DD_ALGO_DD_VALU = 1
DD_ALGO_SLICES_BF16 = 2
DD_ALGO_SLICES_F16 = 3
DD_ALGO_SLICES_I8 = 4
DD_ALGO_SIMPLE_UNFUSED = 5
DD_ALGO_CASCADE_ON_LOAD = 6
DD_SCALING_GLOBAL = 0
DD_SCALING_PANEL = 1
DD_SCALING_BALANCE = 2
DD_NOALLOC_SCRATCH_BYTES = 128 << 20
DD_TILE_AUTO = 0
DD_TILE_64x64 = 1
DD_TILE_32x64 = 2
DD_TILE_64x32 = 3

EXPORTED = ("dd_gemm", "dd_gemm_workspace_size", "dd_gemm_ex", "dd_cascade_split", "dd_slices_split", "dd_dot",
            "dd_scal", "dd_batched_plan_create", "dd_gemm_batched_exec", "dd_batched_plan_tune",
            "dd_batched_plan_schedule", "dd_batched_plan_info", "dd_batched_plan_destroy",
            "dd_gemm_batched", "dd_profile_enable", "dd_phase_times", "dd_status_string", "dd_version",
            "td_gemm_workspace_size", "td_gemm_ex", "dd_gemm_noalloc", "dd_add", "dd_tune",
            "dd_gemm_batched_workspace_size")


class dd_gemm_opts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("kc", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("slices", ctypes.c_int32), ("slice_bits", ctypes.c_int32),
                ("scaling", ctypes.c_int32), ("flags_out", ctypes.c_void_p), ("use_tuned", ctypes.c_int32)]


class DDError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: status %d (%s)" % (where, status, dd_status_string(status)))


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libddgemm.so is not built: run `python -c 'import __graft_entry__ as g; "
                               "g.build()'` (hipcc, gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, i32, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.dd_gemm.argtypes = [i64, i64, i64, vp, vp, i64, vp, vp, i64, vp, vp, i64, vp]
        L.dd_gemm.restype = i32
        L.dd_gemm_workspace_size.argtypes = [i32, i32, i64, i64, i64, ctypes.POINTER(dd_gemm_opts)]
        L.dd_gemm_workspace_size.restype = sz
        L.dd_gemm_ex.argtypes = [i32, i32, i64, i64, i64, vp, vp, i64, vp, vp, i64, vp, vp, i64,
                                 vp, sz, ctypes.POINTER(dd_gemm_opts), vp]
        L.dd_gemm_ex.restype = i32
        L.dd_cascade_split.argtypes = [i32, i32, i64, i64, vp, vp, i64, i32, vp, vp, vp]
        L.dd_cascade_split.restype = i32
        L.dd_slices_split.argtypes = [i32, i32, i64, i64, vp, vp, i64, i32, i32, i32, vp, vp, vp]
        L.dd_slices_split.restype = i32
        L.dd_dot.argtypes = [i64, vp, vp, i64, vp, vp, i64, vp, vp]
        L.dd_dot.restype = i32
        L.dd_scal.argtypes = [i64, vp, vp, vp, i64, vp, vp, i64, vp]
        L.dd_scal.restype = i32
        L.dd_add.argtypes = [i64, vp, vp, i64, vp, vp, i64, vp, vp, i64, vp]
        L.dd_add.restype = i32
        pi64 = ctypes.POINTER(ctypes.c_int64)
        L.dd_batched_plan_create.argtypes = [i32, pi64, pi64, pi64, pi64, pi64, pi64,
                                             ctypes.POINTER(dd_gemm_opts), ctypes.POINTER(vp)]
        L.dd_batched_plan_create.restype = i32
        L.dd_gemm_batched_exec.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.dd_gemm_batched_exec.restype = i32
        L.dd_batched_plan_tune.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp]
        L.dd_batched_plan_tune.restype = i32
        L.dd_batched_plan_schedule.argtypes = [vp, i32, i32, i32, vp]
        L.dd_batched_plan_schedule.restype = i32
        L.dd_batched_plan_info.argtypes = [vp, pi64, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                           ctypes.POINTER(i32), ctypes.POINTER(sz)]
        L.dd_batched_plan_info.restype = i32
        L.dd_batched_plan_destroy.argtypes = [vp]
        L.dd_batched_plan_destroy.restype = i32
        L.dd_gemm_batched.argtypes = [i32, pi64, pi64, pi64, vp, vp, pi64, vp, vp, pi64, vp, vp, pi64,
                                      vp, sz, ctypes.POINTER(dd_gemm_opts), vp]
        L.dd_gemm_batched.restype = i32
        L.dd_gemm_batched_workspace_size.argtypes = [i32, pi64, pi64, pi64, ctypes.POINTER(dd_gemm_opts)]
        L.dd_gemm_batched_workspace_size.restype = sz
        L.dd_profile_enable.argtypes = [i32]
        L.dd_profile_enable.restype = i32
        L.dd_phase_times.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
        L.dd_phase_times.restype = i32
        L.dd_status_string.argtypes = [i32]
        L.dd_status_string.restype = ctypes.c_char_p
        L.dd_version.argtypes = []
        L.dd_version.restype = i32
        L.td_gemm_workspace_size.argtypes = [i32, i32, i64, i64, i64, i32]
        L.td_gemm_workspace_size.restype = sz
        L.td_gemm_ex.argtypes = [i32, i32, i64, i64, i64, vp, vp, vp, i64, vp, vp, vp, i64, vp, vp, vp, i64,
                                 vp, sz, i32, vp]
        L.td_gemm_ex.restype = i32
        L.dd_gemm_noalloc.argtypes = [i32, i32, i64, i64, i64, vp, vp, i64, vp, vp, i64, vp, vp, i64,
                                      ctypes.POINTER(dd_gemm_opts), vp]
        L.dd_gemm_noalloc.restype = i32
        L.dd_tune.argtypes = [i32, pi64, pi64, pi64, ctypes.POINTER(dd_gemm_opts), i32, ctypes.POINTER(i32), vp]
        L.dd_tune.restype = i32
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, dd_gemm_opts):
        return ctypes.byref(opts)
    o = dd_gemm_opts()
    for key, val in dict(opts).items():
        setattr(o, key, _ptr(val) if key == "flags_out" else int(val))
    return ctypes.byref(o)


# ------------------------------------------------------------ the C entry points
def dd_status_string(status: int) -> str:
    return lib().dd_status_string(int(status)).decode()


def dd_version() -> int:
    return int(lib().dd_version())


def dd_gemm(m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc, stream=None) -> int:
    return int(lib().dd_gemm(m, n, k, _ptr(A_hi), _ptr(A_lo), lda, _ptr(B_hi), _ptr(B_lo), ldb,
                             _ptr(C_hi), _ptr(C_lo), ldc, _stream(stream)))


def dd_gemm_workspace_size(transa, transb, m, n, k, opts=None) -> int:
    return int(lib().dd_gemm_workspace_size(int(transa), int(transb), m, n, k, _opts(opts)))


def dd_gemm_ex(transa, transb, m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc,
               workspace=None, ws_bytes=0, opts=None, stream=None) -> int:
    return int(lib().dd_gemm_ex(int(transa), int(transb), m, n, k, _ptr(A_hi), _ptr(A_lo), lda,
                                _ptr(B_hi), _ptr(B_lo), ldb, _ptr(C_hi), _ptr(C_lo), ldc,
                                _ptr(workspace), int(ws_bytes), _opts(opts), _stream(stream)))


def dd_gemm_noalloc(transa, transb, m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc,
                    opts=None, stream=None) -> int:
    return int(lib().dd_gemm_noalloc(int(transa), int(transb), m, n, k, _ptr(A_hi), _ptr(A_lo), lda,
                                     _ptr(B_hi), _ptr(B_lo), ldb, _ptr(C_hi), _ptr(C_lo), ldc,
                                     _opts(opts), _stream(stream)))


def td_gemm_workspace_size(transa, transb, m, n, k, kc=0) -> int:
    return int(lib().td_gemm_workspace_size(int(transa), int(transb), m, n, k, int(kc)))


def td_gemm_ex(transa, transb, m, n, k, A0, A1, A2, lda, B0, B1, B2, ldb, C0, C1, C2, ldc,
               workspace=None, ws_bytes=0, kc=0, stream=None) -> int:
    return int(lib().td_gemm_ex(int(transa), int(transb), m, n, k, _ptr(A0), _ptr(A1), _ptr(A2), lda,
                                _ptr(B0), _ptr(B1), _ptr(B2), ldb, _ptr(C0), _ptr(C1), _ptr(C2), ldc,
                                _ptr(workspace), int(ws_bytes), int(kc), _stream(stream)))


def dd_cascade_split(side, trans, rows, cols, X_hi, X_lo, ldx, kc, exps, planes, stream=None) -> int:
    return int(lib().dd_cascade_split(int(side), int(trans), rows, cols, _ptr(X_hi), _ptr(X_lo), ldx,
                                      int(kc), _ptr(exps), _ptr(planes), _stream(stream)))


def dd_slices_split(side, trans, rows, cols, X_hi, X_lo, ldx, fmt, slices, slice_bits, exps, out,
                    stream=None) -> int:
    return int(lib().dd_slices_split(int(side), int(trans), rows, cols, _ptr(X_hi), _ptr(X_lo), ldx, int(fmt),
                                     int(slices), int(slice_bits), _ptr(exps), _ptr(out), _stream(stream)))


def dd_dot(n, x_hi, x_lo, incx, y_hi, y_lo, incy, result, stream=None) -> int:
    return int(lib().dd_dot(n, _ptr(x_hi), _ptr(x_lo), incx, _ptr(y_hi), _ptr(y_lo), incy, _ptr(result),
                            _stream(stream)))


def dd_scal(n, alpha, x_hi, x_lo, incx, y_hi, y_lo, incy, stream=None) -> int:
    """``alpha``: device memory of two doubles (a tensor or a pointer)."""
    return int(lib().dd_scal(n, _ptr(alpha), _ptr(x_hi), _ptr(x_lo), incx,
                             _ptr(y_hi), _ptr(y_lo), incy, _stream(stream)))


def dd_add(n, x_hi, x_lo, incx, y_hi, y_lo, incy, z_hi, z_lo, incz, stream=None) -> int:
    return int(lib().dd_add(n, _ptr(x_hi), _ptr(x_lo), incx, _ptr(y_hi), _ptr(y_lo), incy,
                            _ptr(z_hi), _ptr(z_lo), incz, _stream(stream)))


def _i64arr(v):
    arr = (ctypes.c_int64 * max(1, len(v)))(*[int(x) for x in v])
    return arr


def dd_batched_plan_create(count, m, n, k, lda, ldb, ldc, opts=None):
    """Returns ``(status, plan)`` (plan is an opaque integer handle)."""
    plan = ctypes.c_void_p()
    st = int(lib().dd_batched_plan_create(int(count), _i64arr(m), _i64arr(n), _i64arr(k), _i64arr(lda),
                                          _i64arr(ldb), _i64arr(ldc), _opts(opts), ctypes.byref(plan)))
    return st, plan.value


def dd_gemm_batched_exec(plan, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, stream=None) -> int:
    return int(lib().dd_gemm_batched_exec(plan, _ptr(A_hi), _ptr(A_lo), _ptr(B_hi), _ptr(B_lo),
                                          _ptr(C_hi), _ptr(C_lo), _stream(stream)))


def dd_batched_plan_tune(plan, A_hi, A_lo, B_hi, B_lo, C_hi, C_lo, repeats=3, stream=None) -> int:
    return int(lib().dd_batched_plan_tune(plan, _ptr(A_hi), _ptr(A_lo), _ptr(B_hi), _ptr(B_lo),
                                          _ptr(C_hi), _ptr(C_lo), int(repeats), _stream(stream)))


def dd_batched_plan_schedule(plan, dynamic, lpt, tile_policy=0, stream=None) -> int:
    return int(lib().dd_batched_plan_schedule(plan, int(dynamic), int(lpt), int(tile_policy), _stream(stream)))


def dd_batched_plan_info(plan):
    """Returns ``(status, ntiles, dynamic, lpt, tile_policy, device_bytes)``."""
    nt, dy, lp, tp, nb = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    st = int(lib().dd_batched_plan_info(plan, ctypes.byref(nt), ctypes.byref(dy), ctypes.byref(lp),
                                        ctypes.byref(tp), ctypes.byref(nb)))
    return st, nt.value, dy.value, lp.value, tp.value, nb.value


def dd_tune(m, n, k, opts=None, repeats=3, stream=None):
    """Tile-shape tuner over the shapes (lists m, n, k); returns ``(status, shapes)``."""
    count = len(m)
    shapes = (ctypes.c_int32 * max(count, 1))()
    st = int(lib().dd_tune(count, _i64arr(m), _i64arr(n), _i64arr(k), _opts(opts), int(repeats), shapes,
                           _stream(stream)))
    return st, [int(shapes[i]) for i in range(count)]


def dd_batched_plan_destroy(plan) -> int:
    return int(lib().dd_batched_plan_destroy(plan))


def dd_gemm_batched(count, m, n, k, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc, workspace=None,
                    ws_bytes=0, opts=None, stream=None) -> int:
    return int(lib().dd_gemm_batched(int(count), _i64arr(m), _i64arr(n), _i64arr(k), _ptr(A_hi), _ptr(A_lo),
                                     _i64arr(lda), _ptr(B_hi), _ptr(B_lo), _i64arr(ldb), _ptr(C_hi),
                                     _ptr(C_lo), _i64arr(ldc), _ptr(workspace), int(ws_bytes), _opts(opts),
                                     _stream(stream)))


def dd_gemm_batched_workspace_size(count, m, n, k, opts=None) -> int:
    return int(lib().dd_gemm_batched_workspace_size(int(count), _i64arr(m), _i64arr(n), _i64arr(k),
                                                    _opts(opts)))


def dd_profile_enable(enable) -> int:
    return int(lib().dd_profile_enable(int(bool(enable))))


def dd_phase_times():
    """Returns ``(status, split_ms, product_ms, calls)`` summed since the last call."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    st = int(lib().dd_phase_times(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return st, a.value, b.value, int(c.value)


def check(status: int, where: str = "ddgemm") -> None:
    if status != DD_OK:
        raise DDError(status, where)


# ------------------------------------------------------------ layout helpers
def colmajor_to_device(a, device="cuda"):
    """numpy (rows x cols, any order) -> contiguous torch tensor (cols, rows) on ``device``."""
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).to(device)


def colmajor_from_device(t):
    """Inverse of :func:`colmajor_to_device`: a Fortran-ordered numpy array."""
    import numpy as np
    return np.asfortranarray(t.detach().cpu().numpy().T)
