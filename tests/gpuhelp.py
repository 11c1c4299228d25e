"""Helpers shared by the GPU tests: upload seeded problems, run the C ABI,
and the tolerances the results are held to."""
from __future__ import annotations

import sys

import numpy as np

from paper_2303_04353_amd import ddgemm as dg


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def up(x):
    return dg.colmajor_to_device(x)


def down(t):
    return dg.colmajor_from_device(t)


def run_gemm(A, B, C, *, transa=False, transb=False, algo=dg.DD_ALGO_CASCADE_F64, kc=0,
             plain=False, slices=0, slice_bits=0, scaling=0):
    """op(A) op(B) + C on the GPU through the C ABI; A, B, C are numpy (hi, lo)
    pairs as stored.  Returns numpy (hi, lo)."""
    import torch
    Ah, Al = up(A[0]), up(A[1])
    Bh, Bl = up(B[0]), up(B[1])
    Ch, Cl = up(C[0]), up(C[1])
    m = A[0].shape[1] if transa else A[0].shape[0]
    k = A[0].shape[0] if transa else A[0].shape[1]
    n = B[0].shape[0] if transb else B[0].shape[1]
    lda, ldb, ldc = max(1, A[0].shape[0]), max(1, B[0].shape[0]), max(1, C[0].shape[0])
    if plain:
        assert not transa and not transb and algo == dg.DD_ALGO_CASCADE_F64 and kc == 0 and scaling == 0
        st = dg.dd_gemm(m, n, k, Ah, Al, lda, Bh, Bl, ldb, Ch, Cl, ldc)
    else:
        st = dg.dd_gemm_ex(int(transa), int(transb), m, n, k, Ah, Al, lda, Bh, Bl, ldb, Ch, Cl, ldc,
                           opts={"algo": algo, "kc": kc, "slices": slices, "slice_bits": slice_bits,
                                 "scaling": scaling})
    dg.check(st, "dd_gemm_ex")
    torch.cuda.synchronize()
    return down(Ch), down(Cl)


def dd_diff(G, O):
    """|G - O| as FP64 for FP64x2 pairs (hi words agree to within a few ulps)."""
    return np.abs((G[0] - O[0]) + (G[1] - O[1]))


def fp64x2_tolerance(A, B, k):
    """64 k 2^-104 (|A||B|)_ij with |A||B| from the high words in FP64."""
    AB = np.abs(np.asarray(A[0])) @ np.abs(np.asarray(B[0]))
    return 64.0 * max(k, 1) * 2.0 ** -104 * AB


def cascade_order_bound(A, B, O, k, kc):
    """Two cascades that differ only in the summation order of bin 3-6 agree to
    within this bound (per entry).  Each bin 3-6 sum has 4*kcb terms of size
    <= 2 sigma_3 after scaling, so two orders differ by <= 64 kcb^2 2^-53
    sigma_3 per block; the FP64x2 combine then adds a few 2^-106 relative."""
    from oracle import cascade as cz  # tests only
    kce = min(kc, k)
    c = cz.split_widths(kce)
    D2 = sum(c)
    e = cz.exponents(A[0], axis=1).astype(np.int64)
    f = cz.exponents(B[0], axis=0).astype(np.int64)
    scale = np.ldexp(1.0, e[:, None] + f[None, :])
    nb = -(-k // kce)
    AB = np.abs(np.asarray(A[0])) @ np.abs(np.asarray(B[0]))
    return (scale * 64.0 * kce * k * 2.0 ** -(53 + D2)
            + 8 * nb * 2.0 ** -106 * AB + 2.0 ** -103 * np.abs(O[0]))


def panel_order_bound(A, B, O, k, kc):
    """cascade_order_bound with Sigma and T per rank-kc panel: each block's
    bin 3-6 order difference is bounded at that panel's scale, so the sum is
    bounded by the largest panel scale times the whole-k term."""
    from oracle import cascade as cz  # tests only
    kce = min(kc, k)
    c = cz.split_widths(kce)
    D2 = sum(c)
    top = None
    for p0 in range(0, k, kce):
        e = cz.exponents(A[0][:, p0:p0 + kce], axis=1).astype(np.int64)
        f = cz.exponents(B[0][p0:p0 + kce, :], axis=0).astype(np.int64)
        s = e[:, None] + f[None, :]
        top = s if top is None else np.maximum(top, s)
    nb = -(-k // kce)
    AB = np.abs(np.asarray(A[0])) @ np.abs(np.asarray(B[0]))
    return (np.ldexp(1.0, top) * 64.0 * kce * k * 2.0 ** -(53 + D2)
            + 8 * nb * 2.0 ** -106 * AB + 2.0 ** -103 * np.abs(O[0]))
