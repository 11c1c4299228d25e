"""dd_gemm / dd_gemm_ex with the library's cached workspace under HIP graph
capture (GPU).

A captured call takes the stream's cached buffer if it is large enough; the
buffer is then never freed, so replays stay bit-identical to the eager call
after later calls on the same stream have grown the cache.  With a cache too
small, a captured call returns DD_ERR_WORKSPACE and launches nothing."""
import ctypes

import numpy as np
import pytest

from oracle.cascade import cascade_gemm
from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import make_problem
from tests.gpuhelp import cascade_order_bound, dd_diff, down, log, up

pytestmark = pytest.mark.gpu


def _upload(P):
    return [up(x) for x in (*P["A"], *P["B"], *P["C"])]


def test_captured_call_survives_cache_growth():
    import torch
    m, n, k = 150, 97, 300
    log(f"capture: dd_gemm {m}x{n}x{k}, then growth by a 512^3 call between replays")
    P = make_problem(m, n, k, cfg=41)
    Ah, Al, Bh, Bl, C0h, C0l = _upload(P)
    Big = make_problem(512, 512, 512, cfg=42)
    bAh, bAl, bBh, bBl, bCh, bCl = _upload(Big)
    s = torch.cuda.Stream()
    Ch, Cl = C0h.clone(), C0l.clone()
    with torch.cuda.stream(s):
        # the eager call sizes this stream's cache for the problem
        dg.check(dg.dd_gemm(m, n, k, Ah, Al, m, Bh, Bl, k, Ch, Cl, m, stream=s), "dd_gemm")
    torch.cuda.synchronize()
    eager = (down(Ch), down(Cl))
    # the eager result is the cascade's, within the bound of its summation order
    O = cascade_gemm(P["A"], P["B"], P["C"], kc=256)
    assert np.all(dd_diff(eager, O) <= cascade_order_bound(P["A"], P["B"], O, k, 256))

    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            dg.check(dg.dd_gemm(m, n, k, Ah, Al, m, Bh, Bl, k, Ch, Cl, m, stream=s), "captured dd_gemm")
    torch.cuda.synchronize()
    for r in range(4):
        Ch.copy_(C0h)
        Cl.copy_(C0l)
        x = torch.randn(500, 500, device="cuda", dtype=torch.float64)   # eager work between replays
        (x @ x).sum().item()
        if r == 1:
            # a larger call on the same stream grows its cache past the captured buffer
            with torch.cuda.stream(s):
                dg.check(dg.dd_gemm(512, 512, 512, bAh, bAl, 512, bBh, bBl, 512, bCh, bCl, 512, stream=s),
                         "dd_gemm 512")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (down(Ch), down(Cl))
        assert np.array_equal(got[0], eager[0]) and np.array_equal(got[1], eager[1]), r
    del g


def test_capture_with_a_cold_cache_is_refused():
    import torch
    m, n, k = 64, 64, 64
    log("capture: dd_gemm_ex on a fresh stream (no cached workspace) under capture")
    P = make_problem(m, n, k, cfg=43)
    Ah, Al, Bh, Bl, Ch, Cl = _upload(P)
    C_before = (down(Ch), down(Cl))
    # a stream of its own (torch's streams come from a pool that earlier calls
    # may have used, with a cache already sized)
    hip = ctypes.CDLL("libamdhip64.so")
    raw = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(raw)) == 0
    try:
        s = torch.cuda.ExternalStream(raw.value)
        x = torch.zeros(16, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                st = dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ch, Cl, m, stream=s)
                x.add_(1.0)   # the graph holds this op only
        torch.cuda.synchronize()
        assert st == dg.DD_ERR_WORKSPACE
        g.replay()
        torch.cuda.synchronize()
        assert float(x.sum()) == 16.0
        got = (down(Ch), down(Cl))
        assert np.array_equal(got[0], C_before[0]) and np.array_equal(got[1], C_before[1])
        del g
    finally:
        torch.cuda.synchronize()
        hip.hipStreamDestroy(raw)
