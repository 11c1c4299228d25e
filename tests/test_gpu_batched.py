"""GPU checks of the batched persistent cascade (C ABI).

* every problem of a batch is bit-identical to a single dd_gemm call (same
  packed planes, same per-tile arithmetic), for every schedule;
* the uneven batch (512 problems, m, n, k log-uniform in [32, 1024]) against
  the FP64x2 oracle on sampled entries of every problem;
* a HIP graph of one execution, replayed several times with eager work in
  between, reproduces the eager result every time;
* the tuner picks a schedule and records it in the cache file;
* the one-shot call with a caller workspace: bit-identical to single calls,
  a workspace too small refused, graph capture once its shapes are known;
* cancellation flags of a batch: every problem's bitmap equal to its single
  call's.
"""
import os

import numpy as np
import pytest

from oracle.ref import dd_gemm_ref_entries
from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import batched_shapes, make_problem
from tests.gpuhelp import log, up

pytestmark = pytest.mark.gpu


class Batch:
    """Device copies of a list of problems plus the pointer arrays."""

    def __init__(self, shapes, cfg=30, prepare=None):
        import torch
        self.shapes = shapes
        self.P = [make_problem(m, n, k, cfg=cfg, salt=i) for i, (m, n, k) in enumerate(shapes)]
        if prepare:
            for i, p in enumerate(self.P):
                prepare(i, p)
        self.A = [(up(p["A"][0]), up(p["A"][1])) for p in self.P]
        self.B = [(up(p["B"][0]), up(p["B"][1])) for p in self.P]
        self.C0 = [(up(p["C"][0]), up(p["C"][1])) for p in self.P]
        self.C = [(c[0].clone(), c[1].clone()) for c in self.C0]
        ptrs = lambda lst, w: torch.tensor([t[w].data_ptr() for t in lst], dtype=torch.int64, device="cuda")
        self.pA = (ptrs(self.A, 0), ptrs(self.A, 1))
        self.pB = (ptrs(self.B, 0), ptrs(self.B, 1))
        self.pC = (ptrs(self.C, 0), ptrs(self.C, 1))
        self.m = [s[0] for s in shapes]
        self.n = [s[1] for s in shapes]
        self.k = [s[2] for s in shapes]
        self.lda = [max(1, s[0]) for s in shapes]
        self.ldb = [max(1, s[2]) for s in shapes]
        self.ldc = [max(1, s[0]) for s in shapes]

    def reset(self):
        for c, c0 in zip(self.C, self.C0):
            c[0].copy_(c0[0])
            c[1].copy_(c0[1])

    def plan(self, opts=None):
        st, plan = dg.dd_batched_plan_create(len(self.shapes), self.m, self.n, self.k, self.lda, self.ldb,
                                             self.ldc, opts)
        dg.check(st, "dd_batched_plan_create")
        return plan

    def exec(self, plan):
        dg.check(dg.dd_gemm_batched_exec(plan, self.pA[0], self.pA[1], self.pB[0], self.pB[1],
                                         self.pC[0], self.pC[1]), "dd_gemm_batched_exec")

    def results(self):
        return [(c[0].cpu().numpy().copy(), c[1].cpu().numpy().copy()) for c in self.C]

    def singles(self, opts=None):
        import torch
        out = []
        for i, (m, n, k) in enumerate(self.shapes):
            ch, cl = self.C0[i][0].clone(), self.C0[i][1].clone()
            st = dg.dd_gemm_ex(0, 0, m, n, k, self.A[i][0], self.A[i][1], self.lda[i], self.B[i][0],
                               self.B[i][1], self.ldb[i], ch, cl, self.ldc[i], opts=opts)
            dg.check(st, "dd_gemm_ex")
            out.append((ch, cl))
        torch.cuda.synchronize()
        return [(c[0].cpu().numpy(), c[1].cpu().numpy()) for c in out]


SMALL = [(37, 50, 300), (1, 1, 1), (64, 64, 64), (0, 5, 7), (5, 0, 7), (6, 9, 0), (130, 70, 1000),
         (17, 200, 33), (128, 3, 257), (65, 65, 65), (200, 128, 520), (3, 3, 3)]


# shapes where 32 x 64 or 64 x 32 tiles cut the padding, and where they do not
MIXED = SMALL + [(80, 200, 300), (200, 90, 260), (33, 70, 257), (96, 96, 40), (160, 30, 600), (20, 150, 1)]


@pytest.mark.parametrize("kc", [0, 128, 20])
def test_batch_equals_single_calls_bitwise_for_every_schedule_and_tile_policy(kc):
    import torch
    b = Batch(MIXED)
    opts = {"kc": kc}
    want = b.singles(opts)
    plan = b.plan(opts)
    try:
        ntiles = {}
        for policy in (0, 1, 2):
            for dyn in (1, 0):
                for lpt in (1, 0):
                    log(f"batched small kc={kc} policy={policy} dynamic={dyn} lpt={lpt}")
                    dg.check(dg.dd_batched_plan_schedule(plan, dyn, lpt, policy))
                    b.reset()
                    b.exec(plan)
                    torch.cuda.synchronize()
                    for i, (g, w) in enumerate(zip(b.results(), want)):
                        assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), (i, policy, dyn, lpt)
            st, nt, _, _, tp, _ = dg.dd_batched_plan_info(plan)
            assert st == 0 and tp == policy
            ntiles[policy] = nt
        # smaller tiles where they cut padding: more (smaller) tiles under policies 1 and 2
        assert ntiles[0] < ntiles[1] <= ntiles[2]
    finally:
        dg.dd_batched_plan_destroy(plan)


def test_batch_with_a_long_inner_dimension_equals_single_calls():
    """One problem of 513 rank-256 blocks among small ones: the persistent
    kernel's tiles of it take far longer than the rest (LPT puts them
    first); every problem still equals its single call bit for bit."""
    import torch
    shapes = [(64, 64, 64), (70, 33, (1 << 17) + 5), (1, 1, 1), (130, 70, 1000), (33, 96, 300)]
    log(f"batched long k: {shapes}")
    b = Batch(shapes, cfg=34)
    want = b.singles()
    plan = b.plan()
    try:
        for dyn in (1, 0):
            dg.check(dg.dd_batched_plan_schedule(plan, dyn, 1, 2))
            b.reset()
            b.exec(plan)
            torch.cuda.synchronize()
            for i, (g, w) in enumerate(zip(b.results(), want)):
                assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), (i, dyn)
    finally:
        dg.dd_batched_plan_destroy(plan)


def test_batch_beyond_the_buffer_load_range_equals_single_calls():
    """A problem with k = 2^20 + 3, whose 64 x 64 tiles' packed blocks span
    more than the 2 GiB of the buffer-load form, makes the plan stage every
    tile through 64-bit global addresses; every problem still equals its
    single call (which stages the small ones through buffer loads) bit for
    bit."""
    import torch
    shapes = [(20, 33, (1 << 20) + 3), (64, 64, 64), (130, 70, 1000), (5, 40, 9)]
    log(f"batched global-address staging: {shapes}")
    b = Batch(shapes, cfg=35)
    want = b.singles()
    plan = b.plan()
    try:
        b.reset()
        b.exec(plan)
        torch.cuda.synchronize()
        for i, (g, w) in enumerate(zip(b.results(), want)):
            assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), i
    finally:
        dg.dd_batched_plan_destroy(plan)


def test_one_shot_entry_point():
    import torch
    b = Batch(SMALL[:6], cfg=31)
    want = b.singles()
    st = dg.dd_gemm_batched(len(b.shapes), b.m, b.n, b.k, b.pA[0], b.pA[1], b.lda, b.pB[0], b.pB[1], b.ldb,
                            b.pC[0], b.pC[1], b.ldc)
    dg.check(st, "dd_gemm_batched")
    torch.cuda.synchronize()
    for g, w in zip(b.results(), want):
        assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1])


def _one_shot(b, ws, nbytes, stream=None, opts=None):
    return dg.dd_gemm_batched(len(b.shapes), b.m, b.n, b.k, b.pA[0], b.pA[1], b.lda, b.pB[0], b.pB[1], b.ldb,
                              b.pC[0], b.pC[1], b.ldc, workspace=ws, ws_bytes=nbytes, opts=opts, stream=stream)


@pytest.mark.parametrize("kc", [0, 128])
def test_one_shot_with_caller_workspace(kc):
    import torch
    log(f"batched one-shot with a caller workspace, kc={kc}")
    b = Batch(MIXED, cfg=34)
    opts = {"kc": kc}
    want = b.singles(opts)
    need = dg.dd_gemm_batched_workspace_size(len(b.shapes), b.m, b.n, b.k, opts)
    assert need > 256
    # the workspace arrives full of junk: the call must clear what it uses
    ws = torch.full((need // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")
    # too small: refused, C untouched
    assert _one_shot(b, ws, need - 8, opts=opts) == dg.DD_ERR_WORKSPACE
    torch.cuda.synchronize()
    for g, c0 in zip(b.results(), b.C0):
        assert np.array_equal(g[0], c0[0].cpu().numpy()) and np.array_equal(g[1], c0[1].cpu().numpy())
    for r in range(2):   # the second call takes the kept tables
        b.reset()
        dg.check(_one_shot(b, ws, need, opts=opts), "dd_gemm_batched")
        torch.cuda.synchronize()
        for i, (g, w) in enumerate(zip(b.results(), want)):
            assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), (r, i)


def test_one_shot_with_workspace_under_graph_capture():
    import ctypes
    import torch
    b = Batch(SMALL, cfg=35)
    want = b.singles()
    need = dg.dd_gemm_batched_workspace_size(len(b.shapes), b.m, b.n, b.k)
    ws = torch.empty(need // 8 + 1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dg.check(_one_shot(b, ws, need, stream=s), "dd_gemm_batched warm-up")   # builds the tables
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            dg.check(_one_shot(b, ws, need, stream=s), "captured dd_gemm_batched")
    torch.cuda.synchronize()
    for r in range(3):
        b.reset()
        x = torch.randn(500, 500, device="cuda", dtype=torch.float64)   # eager work between replays
        (x @ x).sum().item()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (gg, w) in enumerate(zip(b.results(), want)):
            assert np.array_equal(gg[0], w[0]) and np.array_equal(gg[1], w[1]), (r, i)
    del g
    # shapes never seen before cannot be prepared under capture: refused, nothing launched
    b2 = Batch([(40, 41, 42), (43, 44, 45)], cfg=36)
    need2 = dg.dd_gemm_batched_workspace_size(2, b2.m, b2.n, b2.k)
    ws2 = torch.empty(need2 // 8 + 1, dtype=torch.float64, device="cuda")
    hip = ctypes.CDLL("libamdhip64.so")
    raw = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(raw)) == 0
    try:
        s2 = torch.cuda.ExternalStream(raw.value)
        y = torch.zeros(8, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        g2 = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s2):
            with torch.cuda.graph(g2, stream=s2):
                st = _one_shot(b2, ws2, need2, stream=s2)
                y.add_(1.0)   # the graph holds this op only
        torch.cuda.synchronize()
        assert st == dg.DD_ERR_WORKSPACE
        g2.replay()
        torch.cuda.synchronize()
        assert float(y.sum()) == 8.0
        for gg, c0 in zip(b2.results(), b2.C0):
            assert np.array_equal(gg[0], c0[0].cpu().numpy()) and np.array_equal(gg[1], c0[1].cpu().numpy())
        del g2
    finally:
        torch.cuda.synchronize()
        hip.hipStreamDestroy(raw)


def _plant_cancellation(i, P):
    """In every other problem, rows 1 and m-1 of A against columns 0 and n-1
    of B cancel in the leading digits of every block (as in the single-call
    flags test)."""
    A, B = P["A"], P["B"]
    m, k = A[0].shape
    n = B[0].shape[1]
    if i % 2 or m < 2 or n < 1 or k < 2:
        return
    for r in (1, m - 1):
        A[0][r, :] = 0.75
        A[0][r, 1::2] = 0.75 + 2.0 ** -30
        A[1][r, :] = 0.0
    for c in (0, n - 1):
        B[0][:, c] = 0.5
        B[0][1::2, c] = -0.5
        B[1][:, c] = 0.0


def test_batched_cancellation_flags_equal_single_calls():
    import torch
    log("batched cancellation flags")
    b = Batch(MIXED, cfg=37, prepare=_plant_cancellation)
    words = [-(-m * n // 32) for m, n, _ in b.shapes]
    off = np.concatenate([[0], np.cumsum(words)]).astype(np.int64)
    # single calls: each problem's bitmap and result
    want, want_bits = [], []
    for i, (m, n, k) in enumerate(b.shapes):
        ch, cl = b.C0[i][0].clone(), b.C0[i][1].clone()
        fw = torch.full((max(1, words[i]),), -1, dtype=torch.int32, device="cuda")
        dg.check(dg.dd_gemm_ex(0, 0, m, n, k, b.A[i][0], b.A[i][1], b.lda[i], b.B[i][0], b.B[i][1], b.ldb[i],
                               ch, cl, b.ldc[i], opts={"flags_out": fw if words[i] else None}), "dd_gemm_ex")
        torch.cuda.synchronize()
        want.append((ch.cpu().numpy(), cl.cpu().numpy()))
        want_bits.append(fw.cpu().numpy()[:words[i]])
    assert sum(int(np.unpackbits(w.view(np.uint8)).sum()) for w in want_bits) >= 8
    # a plan with flags, then the one-shot call with a caller workspace and flags
    flags = torch.full((int(off[-1]),), -1, dtype=torch.int32, device="cuda")   # the calls zero it
    st, plan = dg.dd_batched_plan_create(len(b.shapes), b.m, b.n, b.k, b.lda, b.ldb, b.ldc, {"flags_out": flags})
    dg.check(st, "dd_batched_plan_create")
    try:
        for policy in (0, 2):
            b.reset()
            flags.fill_(-1)
            dg.check(dg.dd_batched_plan_schedule(plan, 1, 1, policy))
            b.exec(plan)
            torch.cuda.synchronize()
            got = flags.cpu().numpy()
            for i, (g, w) in enumerate(zip(b.results(), want)):
                assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), (policy, i)
                assert np.array_equal(got[off[i]:off[i + 1]], want_bits[i]), (policy, i)
    finally:
        dg.dd_batched_plan_destroy(plan)
    need = dg.dd_gemm_batched_workspace_size(len(b.shapes), b.m, b.n, b.k, {"flags_out": flags})
    ws = torch.empty(need // 8 + 1, dtype=torch.float64, device="cuda")
    b.reset()
    flags.fill_(-1)
    dg.check(_one_shot(b, ws, need, opts={"flags_out": flags}), "dd_gemm_batched flags")
    torch.cuda.synchronize()
    got = flags.cpu().numpy()
    for i, (g, w) in enumerate(zip(b.results(), want)):
        assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), i
        assert np.array_equal(got[off[i]:off[i + 1]], want_bits[i]), i


def test_uneven_batch_512_against_oracle_and_singles():
    import torch
    shapes = batched_shapes(512)
    log(f"uneven batch: {len(shapes)} problems")
    b = Batch(shapes, cfg=3)
    plan = b.plan()
    try:
        b.exec(plan)
        torch.cuda.synchronize()
        got = b.results()
    finally:
        dg.dd_batched_plan_destroy(plan)
    want = b.singles()
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]), i
    rng = np.random.default_rng(9)
    for i, (m, n, k) in enumerate(shapes):
        P = b.P[i]
        I = rng.integers(0, m, 8)
        J = rng.integers(0, n, 8)
        rh, rl, _ = dd_gemm_ref_entries(P["A"], P["B"], P["C"], I, J)
        gh, gl = got[i][0].T[I, J], got[i][1].T[I, J]
        AB = np.array([np.abs(P["A"][0][a]) @ np.abs(P["B"][0][:, c]) for a, c in zip(I, J)])
        assert np.all(np.abs((gh - rh) + (gl - rl)) <= 64 * k * 2.0 ** -104 * AB), i


def test_graph_replays_match_eager():
    import torch
    b = Batch(SMALL, cfg=32)
    plan = b.plan()
    try:
        b.exec(plan)
        torch.cuda.synchronize()
        eager = b.results()
        b.reset()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                dg.check(dg.dd_gemm_batched_exec(plan, b.pA[0], b.pA[1], b.pB[0], b.pB[1], b.pC[0], b.pC[1],
                                                 stream=s))
        torch.cuda.synchronize()
        for r in range(4):
            b.reset()
            x = torch.randn(1000, 1000, device="cuda", dtype=torch.float64)   # eager work between replays
            (x @ x).sum().item()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for i, (gg, w) in enumerate(zip(b.results(), eager)):
                assert np.array_equal(gg[0], w[0]) and np.array_equal(gg[1], w[1]), (r, i)
        del g
    finally:
        dg.dd_batched_plan_destroy(plan)


def test_tuner_records_choice(tmp_path):
    import torch
    os.environ["DDGEMM_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        b = Batch(SMALL[:8], cfg=33)
        plan = b.plan()
        try:
            dg.check(dg.dd_batched_plan_tune(plan, b.pA[0], b.pA[1], b.pB[0], b.pB[1], b.pC[0], b.pC[1], 2))
            st, nt, dyn, lpt, policy, nbytes = dg.dd_batched_plan_info(plan)
            assert st == 0 and nt > 0 and dyn in (0, 1) and lpt in (0, 1) and policy in (0, 1, 2) and nbytes > 0
            words = open(tmp_path / "tune.txt").read().split()
            assert len(words) == 5 and words[0] == "b"
            assert (int(words[2]), int(words[3]), int(words[4])) == (dyn, lpt, policy)
        finally:
            dg.dd_batched_plan_destroy(plan)
        plan2 = b.plan()   # a new plan of the same shapes starts from the recorded choice
        try:
            st, nt2, dyn2, lpt2, policy2, _ = dg.dd_batched_plan_info(plan2)
            assert (dyn2, lpt2, policy2, nt2) == (dyn, lpt, policy, nt)
        finally:
            dg.dd_batched_plan_destroy(plan2)
        torch.cuda.synchronize()
    finally:
        del os.environ["DDGEMM_TUNE_CACHE"]
