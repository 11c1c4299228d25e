"""Benchmark: cascaded FP64x2 GEMM C := A*B + C on one MI355X.

One step = one ``dd_gemm`` over the whole hot path (row/column exponents,
Appendix A split, ten FP64-MFMA products per rank-256 block, FP64x2 combine,
Sigma/T and C added last) at m = n = k = 8192 on seeded synthetic FP64x2
inputs (hi ~ U[-1, 1), lo = hi * 2^-53 * U[-1, 1)), resident in HBM.

Prints ONE JSON line with the effective FP64x2 rate 2mnk/t, the fused
product kernel against the FP64 matrix-core peak (timed live with HIP events
on the GEMM's stream), the software double-double kernel on the same GPU and
inputs, the max / median relative error against the FP64x2 oracle on sampled
entries, and the oracle itself timed on this host's cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6   # MI355X, dense FP64 matrix
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=8192, help="m = n = k")
    ap.add_argument("--shape", default=None, metavar="M,N,K",
                    help="time another shape instead (exploration; not the headline workload)")
    ap.add_argument("--variant", default="uniform", choices=["uniform", "scaled"])
    ap.add_argument("--oracle-seconds", type=float, default=15.0,
                    help="CPU time budget of the sampled oracle run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "cascade_kernel_8192_traffic.json"),
                    help="JSON file with measured HBM bytes per launch of the product kernel "
                         "(used only while the kernel source is unchanged since the measurement)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (512 uneven problems) and differentiation timings")
    ap.add_argument("--slices-only", action="store_true",
                    help="time only the narrow-slice variant at 4096^3 (for profiling it); "
                         "not the headline workload")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the 512 uneven batched GEMMs (for profiling them); not the headline workload")
    ap.add_argument("--sizes-only", action="store_true",
                    help="time only the square-size sweep (128^3 to 8192^3, uniform and ill-scaled)")
    ap.add_argument("--fp64x3-only", action="store_true",
                    help="time only the FP64x3 GEMM at 4096^3 (for profiling it); not the headline workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain elementwise copy of MIB MiB (reads and writes that many "
                         "bytes once), the reference for scaling HBM byte counters")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def bench_batched(torch, dg, stream):
    """512 independent FP64x2 GEMMs, m, n, k log-uniform in [32, 1024]: one
    persistent launch captured in a HIP graph (schedule tuned) against a loop
    of single dd_gemm calls on the same stream."""
    from paper_2303_04353_amd.inputs import batched_shapes, make_problem
    shapes = batched_shapes(512)
    flops = sum(2.0 * m * n * k for m, n, k in shapes)
    A, B, C = [], [], []
    for i, (m, n, k) in enumerate(shapes):
        P = make_problem(m, n, k, cfg=3, salt=i)
        A.append(tuple(dg.colmajor_to_device(x) for x in P["A"]))
        B.append(tuple(dg.colmajor_to_device(x) for x in P["B"]))
        C.append(tuple(dg.colmajor_to_device(x) for x in P["C"]))
    ptr = lambda lst, w: torch.tensor([t[w].data_ptr() for t in lst], dtype=torch.int64, device="cuda")
    pa, pb, pc = (ptr(A, 0), ptr(A, 1)), (ptr(B, 0), ptr(B, 1)), (ptr(C, 0), ptr(C, 1))
    mm, nn, kk = [s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes]
    st, plan = dg.dd_batched_plan_create(len(shapes), mm, nn, kk, mm, kk, mm)
    dg.check(st, "dd_batched_plan_create")
    try:
        dg.check(dg.dd_batched_plan_tune(plan, pa[0], pa[1], pb[0], pb[1], pc[0], pc[1], 3, stream=stream))
        _, ntiles, dyn, lpt, policy, nbytes = dg.dd_batched_plan_info(plan)
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        with torch.cuda.stream(cap):
            with torch.cuda.graph(g, stream=cap):
                dg.check(dg.dd_gemm_batched_exec(plan, pa[0], pa[1], pb[0], pb[1], pc[0], pc[1], stream=cap))
        torch.cuda.synchronize()
        # a few untimed replays first: the clock comes back up after the host-side capture
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        greps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(greps):
                g.replay()
            e1.record(stream)
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / greps
        reps = 5

        def loop():
            for i, (m, n, k) in enumerate(shapes):
                dg.check(dg.dd_gemm(m, n, k, A[i][0], A[i][1], m, B[i][0], B[i][1], k, C[i][0], C[i][1], m,
                                    stream))
        loop()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            loop()
        e1.record(stream)
        torch.cuda.synchronize()
        lms = e0.elapsed_time(e1) / reps
        del g
    finally:
        dg.dd_batched_plan_destroy(plan)
    return {"workload": "512 FP64x2 GEMMs, m, n, k each round(exp(U[ln 32, ln 1024])), uniform inputs",
            "sum_2mnk": flops, "tiles": ntiles,
            "schedule": {"atomic_counter": bool(dyn), "lpt": bool(lpt), "tile_policy": policy},
            "graph_replays_timed": greps, "loop_repeats_timed": reps,
            "graph_ms": round(gms, 3), "graph_gflops": round(flops / (gms * 1e-3) / 1e9, 1),
            "loop_of_dd_gemm_ms": round(lms, 3), "loop_gflops": round(flops / (lms * 1e-3) / 1e9, 1),
            "speedup": round(lms / gms, 2), "plan_device_bytes": nbytes}


PEAK_BF16_MFMA_TFLOPS = 2500.0   # MI355X, dense BF16 / FP16 matrix


SLICES_FORMATS = (("bf16", 8, 14), ("f16", 8, 14), ("i8", 7, 16))   # (format, w, s)
PEAK_I8_MFMA_TOPS = 5000.0       # MI355X, dense INT8 matrix


def bench_slices(torch, dg, stream, n=4096, reps=3):
    """The narrow-slice precision variant at m = n = k = 4096: BF16 and FP16
    slices (w = 8 bits, s = 14 slices, 105 products, FP32 level sums flushed
    to FP64) and INT8 slices (w = 7, s = 16, 136 products, INT32 level sums),
    uniform and ill-scaled inputs.  Returns the timings and, per case, the
    device result's sampled entries for the accuracy check of the
    CPU-baseline leg."""
    from paper_2303_04353_amd.inputs import make_problem, sample_entries
    algos = {"bf16": dg.DD_ALGO_SLICES_BF16, "f16": dg.DD_ALGO_SLICES_F16, "i8": dg.DD_ALGO_SLICES_I8}
    out = {"workload": f"FP64x2 GEMM C := A*B + C, m=n=k={n}, slices s(s+1)/2 products on 32x32x16 "
                       "BF16/FP16 MFMA (exact FP32 level sums, flushed every 4 steps) or 32x32x32 INT8 "
                       "MFMA (exact INT32 level sums)",
           "formats": {f: {"slice_bits": w, "slices": s, "products": s * (s + 1) // 2}
                       for f, w, s in SLICES_FORMATS},
           "cases": {}}
    samples = {}
    I, J = sample_entries(n, n, 4096, seed=13)
    for variant in ("uniform", "scaled"):
        P = make_problem(n, n, n, cfg=2, variant=variant)
        Ah, Al, Bh, Bl, C0h, C0l = (dg.colmajor_to_device(x) for x in (*P["A"], *P["B"], *P["C"]))
        for fmt, w, s in SLICES_FORMATS:
            algo = algos[fmt]
            prods = s * (s + 1) // 2
            opts = {"algo": algo, "slices": s, "slice_bits": w}
            Ch, Cl = C0h.clone(), C0l.clone()
            dg.check(dg.dd_gemm_ex(0, 0, n, n, n, Ah, Al, n, Bh, Bl, n, Ch, Cl, n, opts=opts, stream=stream))
            torch.cuda.synchronize()
            Gh = Ch.T[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy()
            Gl = Cl.T[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy()
            dg.dd_profile_enable(1)
            dg.dd_phase_times()
            t0 = time.perf_counter()
            for _ in range(reps):
                dg.check(dg.dd_gemm_ex(0, 0, n, n, n, Ah, Al, n, Bh, Bl, n, Ch, Cl, n, opts=opts, stream=stream))
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            st, sp, pr, calls = dg.dd_phase_times()
            dg.dd_profile_enable(0)
            pr /= max(calls, 1)
            sp /= max(calls, 1)
            mfma = prods * 2.0 * n ** 3 / (pr * 1e-3) / 1e12
            peak = PEAK_I8_MFMA_TOPS if fmt == "i8" else PEAK_BF16_MFMA_TFLOPS
            out["cases"][f"{fmt}_{variant}"] = {
                "ms": round(ms, 3), "gflops": round(2.0 * n ** 3 / (ms * 1e-3) / 1e9, 1),
                "split_ms": round(sp, 3), "product_ms": round(pr, 3),
                "matrix_tops": round(mfma, 1), "matrix_peak_tops": peak,
                "pct_of_matrix_peak": round(100 * mfma / peak, 1)}
            samples[(fmt, variant)] = (Gh, Gl)
            del Ch, Cl
        samples[("problem", variant)] = P
        del Ah, Al, Bh, Bl, C0h, C0l
    out["vendor_gemm"] = [vendor_narrow_rates(torch, v) for v in (n, 2 * n)]
    return out, samples, (I, J)


def vendor_narrow_rates(torch, n=4096, seconds=0.012):
    """The vendor library's BF16, FP16 and INT8 GEMMs at n^3 (torch.matmul,
    torch._int_mm), launched back to back for about as long as one slices
    product runs, so that the clock settles the way it does under the
    slices kernels.  A reference point for what the matrix cores sustain on
    these formats; it computes nothing of the FP64x2 product."""
    out = {"library": f"torch ({torch.backends.cuda.preferred_blas_library()})", "n": n}
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    for fmt in ("bf16", "f16", "i8"):
        try:
            if fmt == "i8":
                a = torch.randint(-64, 64, (n, n), device="cuda", dtype=torch.int8, generator=g)
                b = torch.randint(-64, 64, (n, n), device="cuda", dtype=torch.int8, generator=g)
                c = torch.empty(n, n, device="cuda", dtype=torch.int32)
                call = lambda: torch._int_mm(a, b, out=c)  # noqa: E731
                peak = PEAK_I8_MFMA_TOPS
            else:
                dt = torch.bfloat16 if fmt == "bf16" else torch.float16
                a = torch.randn(n, n, device="cuda", dtype=dt, generator=g)
                b = torch.randn(n, n, device="cuda", dtype=dt, generator=g)
                c = torch.empty(n, n, device="cuda", dtype=dt)
                call = lambda: torch.matmul(a, b, out=c)  # noqa: E731
                peak = PEAK_BF16_MFMA_TFLOPS
            for _ in range(5):
                call()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            torch.cuda.synchronize()
            reps = max(10, int(seconds * 1e3 / max(e0.elapsed_time(e1), 1e-3)))
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rate = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
            out[fmt] = {"launches": reps, "ms_per_gemm": round(ms, 4), "matrix_tops": round(rate, 1),
                        "pct_of_matrix_peak": round(100 * rate / peak, 1)}
            del a, b, c
        except Exception as exc:   # a format the library does not offer here
            out[fmt] = {"error": f"{type(exc).__name__}: {exc}"[:200]}
    return out


def slices_accuracy(out, samples, IJ, n=4096):
    """Sampled entries of the slices results against the FP64x2 oracle, and
    bit for bit against the slices oracle (CPU-baseline leg)."""
    from oracle.ref import dd_gemm_ref_entries
    from oracle.slices import slices_gemm_entries
    I, J = IJ
    for variant in ("uniform", "scaled"):
        P = samples[("problem", variant)]
        Rh, Rl, _ = dd_gemm_ref_entries(P["A"], P["B"], P["C"], I, J)
        k = 96   # exact slices-oracle entries (each a full split of one row and one column)
        AB = abs_ab_entries(P["A"][0], P["B"][0], I, J)
        for fmt, w, s in SLICES_FORMATS:
            Sh, Sl = slices_gemm_entries(P["A"], P["B"], P["C"], I[:k], J[:k], w=w, s=s, fmt=fmt)
            Gh, Gl = samples[(fmt, variant)]
            diff = np.abs((Gh - Rh) + (Gl - Rl))
            nz = np.abs(Rh) > 0
            rel = diff[nz] / np.abs(Rh[nz])
            normed = diff / AB
            out["cases"][f"{fmt}_{variant}"].update({
                "sampled_entries": int(len(I)), "max_rel_err": float(np.max(rel)),
                "median_rel_err": float(np.median(rel)),
                "max_err_over_absAabsB": float(np.max(normed)),
                "median_err_over_absAabsB": float(np.median(normed)),
                "tolerance_checked_entries": int(len(normed)),
                "within_tolerance": bool(np.all(normed <= 64 * n * 2.0 ** -104)),
                "slices_oracle_entries": k,
                "bitwise_equal_to_slices_oracle": bool(np.array_equal(Gh[:k], Sh) and np.array_equal(Gl[:k], Sl))})


def abs_ab_entries(Ahi, Bhi, I, J, chunk=1 << 16):
    """(|A_hi| |B_hi|)_ij at the positions (I, J): the scale of the tolerance
    64 k 2^-104 (|A||B|)_ij, in FP64.  One host product of the absolute
    values (BLAS on the host cores), then gathered."""
    AB = np.abs(Ahi) @ np.abs(Bhi)
    return np.concatenate([AB[I[c:c + chunk], J[c:c + chunk]] for c in range(0, len(I), chunk)])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_single_thread_rate(n=1024, entries=16384):
    """DD multiply-adds per second of the FP64x2 oracle on one host core, on
    sampled entries of a uniform n^3 problem (each a full length-n dot
    product)."""
    from oracle.ref import dd_gemm_ref_entries
    from paper_2303_04353_amd.inputs import make_problem, sample_entries
    P = make_problem(n, n, n, cfg=1)
    I, J = sample_entries(n, n, entries, seed=23)
    t = time.perf_counter()
    _, _, used = dd_gemm_ref_entries(P["A"], P["B"], P["C"], I, J, threads=1)
    dt = time.perf_counter() - t
    return {"n": n, "entries": entries, "threads": int(used), "dd_mac_per_s": round(entries * n / dt)}


SIZES = ((128, "uniform"), (1024, "uniform"), (1024, "scaled"), (4096, "uniform"), (4096, "scaled"),
         (8192, "scaled"))


def bench_sizes(torch, dg, stream, cpu=True):
    """The square sizes of the performance study (Sec. 5.1 measures square
    m = n = k): dd_gemm at 128^3, 1024^3, 4096^3 (uniform and ill-scaled) and
    8192^3 ill-scaled, timed with events on the GEMM's stream, with the
    product kernel's share (phase events) against the FP64 matrix peak and
    the software double-double kernel beside it up to 4096^3.  With `cpu`,
    the FP64x2 oracle on every entry (128^3, 1024^3) or 4096 seeded entries
    (larger sizes): max and median relative error and error over
    (|A||B|)_ij, the tolerance, and whether the comparator equals the
    oracle there."""
    from oracle.ref import dd_gemm_ref_entries
    from paper_2303_04353_amd.inputs import make_problem, sample_entries
    out = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    for N, variant in SIZES:
        log(f"sizes: {N}^3 {variant}")
        P = make_problem(N, N, N, cfg=1, variant=variant)
        Ah, Al, Bh, Bl, C0h, C0l = (dg.colmajor_to_device(x) for x in (*P["A"], *P["B"], *P["C"]))
        Ch, Cl = C0h.clone(), C0l.clone()
        reps = 50 if N <= 128 else (20 if N <= 1024 else (5 if N <= 4096 else 3))

        def call():
            dg.check(dg.dd_gemm(N, N, N, Ah, Al, N, Bh, Bl, N, Ch, Cl, N, stream), "dd_gemm")
        call()
        call()
        torch.cuda.synchronize()
        dg.dd_profile_enable(1)
        dg.dd_phase_times()
        ms = timed(call, reps)
        st, sp, pr, calls = dg.dd_phase_times()
        dg.dd_profile_enable(0)
        dg.check(st, "dd_phase_times")
        pr, sp = pr / max(calls, 1), sp / max(calls, 1)
        flops, mfma = 2.0 * N ** 3, 20.0 * N ** 3
        case = {"ms": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
                "split_ms": round(sp, 4), "product_ms": round(pr, 4),
                "fp64_mfma_tflops": round(mfma / (pr * 1e-3) / 1e12, 2),
                "pct_of_fp64_mfma_peak": round(100 * mfma / (pr * 1e-3) / 1e12 / PEAK_FP64_MFMA_TFLOPS, 1),
                "algorithmic_gbps": round((16 * 2 * N * N + 32 * N * N) / (ms * 1e-3) / 1e9, 1)}
        Ch.copy_(C0h)
        Cl.copy_(C0l)
        call()
        torch.cuda.synchronize()
        if N <= 1024:
            I, J = (x.ravel() for x in np.meshgrid(np.arange(N), np.arange(N), indexing="ij"))
        else:
            I, J = sample_entries(N, N, 4096, seed=N + 1)
        ti, tj = torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()
        Gh, Gl = Ch.T[ti, tj].cpu().numpy(), Cl.T[ti, tj].cpu().numpy()
        V = None
        if N <= 4096:
            Vh, Vl = C0h.clone(), C0l.clone()
            vopts = {"algo": dg.DD_ALGO_DD_VALU}

            def vcall():
                dg.check(dg.dd_gemm_ex(0, 0, N, N, N, Ah, Al, N, Bh, Bl, N, Vh, Vl, N, opts=vopts, stream=stream))
            vcall()
            torch.cuda.synchronize()
            Vh.copy_(C0h)
            Vl.copy_(C0l)
            vms = timed(vcall, 1)
            V = (Vh.T[ti, tj].cpu().numpy(), Vl.T[ti, tj].cpu().numpy())
            case["comparator_ms"] = round(vms, 4)
            case["comparator_gflops"] = round(flops / (vms * 1e-3) / 1e9, 1)
            del Vh, Vl
        if cpu:
            t = time.perf_counter()
            Rh, Rl, used = dd_gemm_ref_entries(P["A"], P["B"], P["C"], I, J)
            dt = time.perf_counter() - t
            diff = np.abs((Gh - Rh) + (Gl - Rl))
            nz = np.abs(Rh) > 0
            rel = diff[nz] / np.abs(Rh[nz])
            normed = diff / abs_ab_entries(P["A"][0], P["B"][0], I, J)
            case.update({
                "oracle": "every entry" if N <= 1024 else f"{len(I)} seeded entries",
                "oracle_s": round(dt, 3), "oracle_threads": int(used),
                "max_rel_err": float(np.max(rel)), "median_rel_err": float(np.median(rel)),
                "max_err_over_absAabsB": float(np.max(normed)),
                "median_err_over_absAabsB": float(np.median(normed)),
                "tolerance_over_absAabsB": 64 * N * 2.0 ** -104,
                "within_tolerance": bool(np.all(normed <= 64 * N * 2.0 ** -104))})
            if V is not None:
                case["comparator_bitwise_equal_to_oracle"] = bool(np.array_equal(V[0], Rh) and
                                                                  np.array_equal(V[1], Rl))
        out[f"{N}_{variant}"] = case
        del Ah, Al, Bh, Bl, C0h, C0l, Ch, Cl, P
        torch.cuda.empty_cache()
    return out


ACCURACY_WORKLOADS = ("uniform", "wide", "ill-1e-9", "ill-1e-14", "ill-1e-19")
ACCURACY_SIZES = (128, 256, 257, 384)   # ill-conditioned, t = 1e-14, kc = 256


def _accuracy_case(torch, dg, name, n, slices=False):
    """Cascade and FP64x2 comparator (and, with `slices`, the INT8 slices
    variant) on the GPU for one accuracy workload, every entry's relative
    error against the exact product."""
    from oracle.illcond import ill_conditioned
    from oracle.ref import exact_entries
    from paper_2303_04353_amd.inputs import make_problem
    P = (ill_conditioned(n, float(name[4:]), seed=0) if name.startswith("ill")
         else make_problem(n, n, n, cfg=0, variant=name))
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    I, J = I.ravel(), J.ravel()
    dev = [dg.colmajor_to_device(x) for x in (*P["A"], *P["B"])]
    rel, case = {}, {}
    algos = [("cascade", dg.DD_ALGO_CASCADE_F64), ("fp64x2", dg.DD_ALGO_DD_VALU)]
    if slices:
        algos.append(("slices_i8", dg.DD_ALGO_SLICES_I8))
    for label, algo in algos:
        Ch, Cl = dg.colmajor_to_device(P["C"][0]), dg.colmajor_to_device(P["C"][1])
        opts = {"algo": algo}
        flags = None
        if algo == dg.DD_ALGO_CASCADE_F64:
            flags = torch.zeros(((n * n + 31) // 32,), dtype=torch.int32, device="cuda")
            opts["flags_out"] = flags
        dg.check(dg.dd_gemm_ex(0, 0, n, n, n, dev[0], dev[1], n, dev[2], dev[3], n, Ch, Cl, n, opts=opts))
        torch.cuda.synchronize()
        R = dg.colmajor_from_device(Ch), dg.colmajor_from_device(Cl)
        ex, err = exact_entries(P["A"], P["B"], P["C"], I, J, (R[0][I, J], R[1][I, J]))
        rel[label] = np.abs(err) / np.abs(ex)
        case[f"{label}_max_rel_err"] = float(rel[label].max())
        if flags is not None:
            bits = np.unpackbits(flags.cpu().numpy().view(np.uint8), bitorder="little")
            case["cascade_entries_flagged"] = int(bits[:n * n].sum())
    return rel, case


def accuracy_workloads(torch, dg, n=240):
    """The paper's element-wise accuracy study (Sec. 5.2) at n = 240: uniform,
    wide-range and ill-conditioned (t = 1e-9, 1e-14, 1e-19) inputs, the
    cascade, the FP64x2 comparator kernel and the INT8 slices on the GPU, every entry's
    relative error against the exact product; then the largest error by
    problem size around kc = 256, where the cascade starts to accumulate
    several rank-kc blocks in FP64x2 (CPU-baseline leg: the exact reference
    and the generators are test infrastructure)."""
    out = {"n": n, "reference": "exact (expansion arithmetic)", "cases": {}, "by_size_ill_1e-14": {}}
    for name in ACCURACY_WORKLOADS:
        rel, case = _accuracy_case(torch, dg, name, n, slices=True)
        ratio = np.sort(rel["fp64x2"] / np.maximum(rel["cascade"], 1e-300))
        case["frac_cascade_at_least_as_accurate"] = round(float(np.mean(rel["cascade"] <= rel["fp64x2"])), 4)
        case["ratio_fp64x2_over_cascade_quantiles"] = {
            q: float(ratio[min(len(ratio) - 1, int(float(q) * len(ratio)))]) for q in ("0.01", "0.1", "0.5", "0.9")}
        out["cases"][name] = case
    for size in ACCURACY_SIZES:
        _, case = _accuracy_case(torch, dg, "ill-1e-14", size)
        case["ratio_of_max_errors"] = case["fp64x2_max_rel_err"] / max(case["cascade_max_rel_err"], 1e-300)
        out["by_size_ill_1e-14"][str(size)] = case
    return out


def scaling_accuracy(torch, dg, variant, modes, m=512, n=512, k=4096, kc=256):
    """Global Sigma and T against per-panel scaling or diagonal balancing on
    inputs built to need them ('panels': the scale of every row and column
    changes from panel to panel by up to 2^80; 'skewed': column p of A and
    row p of B carry 2^s_p and 2^-s_p, |s_p| <= 40): max error over
    (|A||B| + |C|)_ij against the FP64x2 oracle, and the share of entries
    within the tolerance (CPU-baseline leg: the oracle is test
    infrastructure)."""
    from oracle.ref import dd_gemm_ref
    from paper_2303_04353_amd.inputs import make_problem
    P = make_problem(m, n, k, cfg=3, variant=variant, panel=kc)
    R = dd_gemm_ref(P["A"], P["B"], P["C"])[:2]
    AB = np.abs(P["A"][0]) @ np.abs(P["B"][0]) + np.abs(P["C"][0])
    tol = 64 * k * 2.0 ** -104
    dev = [dg.colmajor_to_device(x) for x in (*P["A"], *P["B"])]
    out = {"workload": f"m={m} n={n} k={k} kc={kc}, '{variant}' inputs", "tolerance_over_absAabsB": tol}
    for name, scaling in modes:
        Ch, Cl = dg.colmajor_to_device(P["C"][0]), dg.colmajor_to_device(P["C"][1])
        dg.check(dg.dd_gemm_ex(0, 0, m, n, k, dev[0], dev[1], m, dev[2], dev[3], k, Ch, Cl, m,
                               opts={"kc": kc, "scaling": scaling}))
        torch.cuda.synchronize()
        G = dg.colmajor_from_device(Ch), dg.colmajor_from_device(Cl)
        r = np.abs((G[0] - R[0]) + (G[1] - R[1])) / AB
        out[name] = {"max_err_over_absAabsB": float(r.max()), "frac_within_tolerance": float(np.mean(r <= tol))}
    return out


def panel_scaling(torch, dg):
    return scaling_accuracy(torch, dg, "panels", (("global", dg.DD_SCALING_GLOBAL), ("panel", dg.DD_SCALING_PANEL)))


def balancing(torch, dg):
    return scaling_accuracy(torch, dg, "skewed", (("global", dg.DD_SCALING_GLOBAL),
                                                  ("balanced", dg.DD_SCALING_BALANCE)))


def bench_td(torch, dg, stream, n=4096, reps=1):
    """FP64x3 (triple-word) GEMM at n^3: average time of td_gemm_ex (maxima,
    split into six packed digit planes, the fused kernel with 21 FP64-MFMA
    products per group of 4 inner indices and a triple-word combine per
    rank-256 block) on seeded three-word operands over `reps` calls.  The
    CPU-baseline leg adds the difference from the FP64x3 oracle
    (td_accuracy)."""
    from paper_2303_04353_amd.inputs import make_problem3
    P = make_problem3(n, n, n, cfg=5)
    Ad = [dg.colmajor_to_device(x) for x in P["A"]]
    Bd = [dg.colmajor_to_device(x) for x in P["B"]]
    C0 = [dg.colmajor_to_device(x) for x in P["C"]]
    Cd = [x.clone() for x in C0]
    dg.check(dg.td_gemm_ex(0, 0, n, n, n, *Ad, n, *Bd, n, *Cd, n, stream=stream))
    torch.cuda.synchronize()
    # sampled entries of this first (untimed) result, for the CPU-baseline leg
    from paper_2303_04353_amd.inputs import sample_entries
    I, J = sample_entries(n, n, 256, seed=17)
    ti, tj = torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()
    samples = [x.T[ti, tj].cpu().numpy() for x in Cd]   # the tensors hold C transposed
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        dg.check(dg.td_gemm_ex(0, 0, n, n, n, *Ad, n, *Bd, n, *Cd, n, stream=stream))
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    mfma = 21 * 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    return {"workload": f"FP64x3 GEMM C := A*B + C, m=n=k={n}, three-word operands (about 159 bits), "
                        "6 FP64 digits, 21 products per group of 4 inner indices in one fused FP64-MFMA kernel, "
                        "triple-word combine per rank-256 block",
            "ms": round(ms, 3), "value": round(2.0 * n ** 3 / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
            "fp64_mfma_tflops_whole_call": round(mfma, 2),
            "pct_of_fp64_mfma_peak_whole_call": round(100 * mfma / PEAK_FP64_MFMA_TFLOPS, 1),
            "_samples": (P, I, J, samples)}


def td_sampled_check(P, I, J, S):
    """Sampled entries S (three word arrays) of the FP64x3 result C + A B at
    positions (I, J) against the oracle, each entry from its row of A and
    column of B alone, within the bound for the tail bin's summation order."""
    from oracle.cascade3 import cascade3_gemm, widths3
    k = P["A"][0].shape[1]
    worst, ok = 0.0, True
    for t, (i, j) in enumerate(zip(I, J)):
        a = tuple(x[i:i + 1, :] for x in P["A"])
        b = tuple(x[:, j:j + 1] for x in P["B"])
        c = tuple(x[i:i + 1, j:j + 1] for x in P["C"])
        o = cascade3_gemm(a, b, c, kc=256)
        d = abs(((S[0][t] - o[0][0, 0]) + (S[1][t] - o[1][0, 0])) + (S[2][t] - o[2][0, 0]))
        ab = float((np.abs(a[0]) @ np.abs(b[0]))[0, 0])
        # tail bins: 6 kc products summed in another order, per block
        ea, eb = np.frexp(np.max(np.abs(a[0])))[1], np.frexp(np.max(np.abs(b[0])))[1]
        bound = (k // 256) * 1024.0 * 256 * 256 * 2.0 ** (int(ea) + int(eb) - 53 - sum(widths3(256))) \
            + 2.0 ** -150 * (abs(o[0][0, 0]) + ab)
        ok &= bool(d <= bound)
        worst = max(worst, d / ab)
    return {"entries": int(len(I)), "max_diff_from_oracle_over_absAabsB": float(worst),
            "within_order_bound": ok}


def td_accuracy(torch, dg, out, n=256):
    """FP64x3 results against the FP64x3 oracle (CPU-baseline leg): every
    entry at n^3, and 256 sampled entries of the timed 4096^3 problem (the
    oracle computes entry (i, j) from row i of A and column j of B alone:
    the powers of two are per row and per column), the latter within the
    bound for the tail bin's summation order."""
    from oracle.cascade3 import cascade3_gemm
    from paper_2303_04353_amd.inputs import make_problem3
    out["check_sampled_4096"] = td_sampled_check(*out.pop("_samples"))
    P = make_problem3(n, n, n, cfg=6)
    Ad = [dg.colmajor_to_device(x) for x in P["A"]]
    Bd = [dg.colmajor_to_device(x) for x in P["B"]]
    Cd = [dg.colmajor_to_device(x) for x in P["C"]]
    dg.check(dg.td_gemm_ex(0, 0, n, n, n, *Ad, n, *Bd, n, *Cd, n))
    torch.cuda.synchronize()
    G = [dg.colmajor_from_device(x) for x in Cd]
    O = cascade3_gemm(P["A"], P["B"], P["C"], kc=256)
    d = np.abs(((G[0] - O[0]) + (G[1] - O[1])) + (G[2] - O[2]))
    AB = np.abs(P["A"][0]) @ np.abs(P["B"][0])
    out["check"] = {"n": n, "max_diff_from_oracle_over_absAabsB": float(np.max(d / AB))}


def bench_autograd(torch):
    """Forward and cascaded backward of L = sum((W2 (W1 X)) o G), W 2048^2, X, G 2048x512."""
    from paper_2303_04353_amd import autograd as ag
    from paper_2303_04353_amd.inputs import make_pair
    n, b = 2048, 512
    mk = lambda shape, seed: ag.dd_from_pair(*[torch.from_numpy(v.copy()) for v in make_pair(shape, seed=seed)]).cuda()
    W1, W2, X, G = mk((n, n), 11), mk((n, n), 12), mk((n, b), 13), mk((n, b), 14)
    gL = torch.tensor([1.0, 0.0], dtype=torch.float64, device="cuda")

    def run():
        w1, w2, x = (t.detach().requires_grad_() for t in (W1, W2, X))
        ag.chain_loss(w1, w2, x, G).backward(gL)
    run()
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flops = 6 * 2.0 * n * n * b
    return {"workload": "L = sum((W2 (W1 X)) o G), W1, W2 2048x2048, X, G 2048x512, forward + backward "
                        "(2 + 4 cascaded GEMMs)", "ms": round(ms, 3), "gflops": round(flops / (ms * 1e-3) / 1e9, 1)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the GEMM shards over output tiles without communication; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_04353_amd import ddgemm as dg
    from paper_2303_04353_amd.inputs import make_problem, sample_entries

    torch.cuda.set_device(0)
    dg.lib()  # fails loudly if the HIP library is missing
    if args.copy_calibration > 0:
        # the reference for scaling HBM byte counters: one elementwise kernel
        # that reads and writes the given size once
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: {nel * 8} bytes read and written by one elementwise kernel")
        del src, dst
    if args.slices_only:
        sres, samples, IJ = bench_slices(torch, dg, torch.cuda.current_stream(), reps=max(1, args.steps))
        if not args.no_cpu_baseline:
            slices_accuracy(sres, samples, IJ)
        print(json.dumps({"slices": sres}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(torch, dg, torch.cuda.current_stream())}), flush=True)
        return
    if args.sizes_only:
        print(json.dumps({"sizes": bench_sizes(torch, dg, torch.cuda.current_stream(),
                                               cpu=not args.no_cpu_baseline)}), flush=True)
        return
    if args.fp64x3_only:
        tres = bench_td(torch, dg, torch.cuda.current_stream(), reps=max(1, args.steps))
        if not args.no_cpu_baseline:
            td_accuracy(torch, dg, tres)
        tres.pop("_samples", None)
        print(json.dumps({"fp64x3": tres}), flush=True)
        return
    N = args.size
    m = n = k = N
    if args.shape:
        m, n, k = (int(v) for v in args.shape.split(","))
    log(f"generating inputs m={m} n={n} k={k} variant={args.variant}")
    P = make_problem(m, n, k, cfg=1, variant=args.variant)
    dev = {key: (dg.colmajor_to_device(v[0]), dg.colmajor_to_device(v[1])) for key, v in P.items()}
    Ah, Al = dev["A"]
    Bh, Bl = dev["B"]
    C0h, C0l = dev["C"]
    Ch, Cl = C0h.clone(), C0l.clone()
    stream = torch.cuda.current_stream()

    def step():
        dg.check(dg.dd_gemm(m, n, k, Ah, Al, m, Bh, Bl, k, Ch, Cl, m, stream), "dd_gemm")

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dg.dd_profile_enable(1)
    dg.dd_phase_times()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, split_ms, prod_ms, calls = dg.dd_phase_times()
    dg.dd_profile_enable(0)
    dg.check(st, "dd_phase_times")
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    flops_eff = 2.0 * m * n * k
    value = flops_eff / (ms_per_step * 1e-3) / 1e9
    prod_avg_ms = prod_ms / max(calls, 1)
    split_avg_ms = split_ms / max(calls, 1)
    mfma_flops = 20.0 * m * n * k
    achieved = mfma_flops / (prod_avg_ms * 1e-3) / 1e12
    log(f"{ms_per_step:.2f} ms/step, {value:.1f} GFLOP/s effective; product kernel {prod_avg_ms:.2f} ms "
        f"({achieved:.2f} TFLOP/s FP64 MFMA), phase one {split_avg_ms:.2f} ms")


    from paper_2303_04353_amd.profiling import load_traffic
    traffic = load_traffic(args.traffic, m, n, k)

    # ---- accuracy on sampled entries: one more GEMM on a fresh copy of C
    Ch.copy_(C0h)
    Cl.copy_(C0l)
    step()
    torch.cuda.synchronize()
    result = {
        "metric": "effective FP64x2 GFLOP/s (2mnk/t) & % FP64 MFMA peak at 8192^3, max rel err vs oracle",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64x2 GEMM C := A*B + C, m={m} n={n} k={k}, {args.variant} "
                               "(hi ~ U[-1,1), lo = hi*2^-53*U[-1,1)), column-major hi/lo planes in HBM",
                   "m": m, "n": n, "k": k, "kc": 256, "algo": "cascade_f64 (10 FP64 MFMA products)",
                   "parallelism": "single GPU"},
        "fp64_mfma_util_pct_of_peak": round(100.0 * (20.0 * m * n * k) / (ms_per_step * 1e-3) / 1e12
                                            / PEAK_FP64_MFMA_TFLOPS, 2),
        "phases_ms": {"split": round(split_avg_ms, 3), "product": round(prod_avg_ms, 3)},
        "roofline": {"bound": "mfma", "kernel": "cascade_kernel",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_MFMA_TFLOPS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "algorithmic": "20*m*n*k FP64 flops per launch (10 products)",
                     # the minimum: A and B as hi/lo planes read once, C read and written
                     "algorithmic_bytes": 16 * (m * k + k * n) + 32 * m * n,
                     # what the kernel must at least read as designed: 4 + 5 packed digit planes, C
                     "packed_plane_bytes": 8 * (4 * m * k + 7 * k * n) + 32 * m * n},
    }
    rf = result["roofline"]
    if traffic is not None:
        rf["traffic_over_algorithmic_bytes"] = round(traffic / rf["algorithmic_bytes"], 2)
        rf["traffic_over_packed_plane_bytes"] = round(traffic / rf["packed_plane_bytes"], 2)
        rf["hbm_gbps"] = round(traffic / (prod_avg_ms * 1e-3) / 1e9, 1)
        rf["hbm_frac"] = round(rf["hbm_gbps"] / PEAK_HBM_GBS, 4)

    I, J = sample_entries(m, n, 1 << 20, seed=7)
    Gh = Ch.T[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy()
    Gl = Cl.T[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy()

    if not args.no_comparator:
        log("software double-double kernel")
        Vh, Vl = C0h.clone(), C0l.clone()
        opts = {"algo": dg.DD_ALGO_DD_VALU}
        dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Vh, Vl, m, opts=opts, stream=stream))
        torch.cuda.synchronize()
        Vh.copy_(C0h)
        Vl.copy_(C0l)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Vh, Vl, m, opts=opts, stream=stream))
        ev1.record(stream)
        torch.cuda.synchronize()
        vms = ev0.elapsed_time(ev1)
        result["comparator"] = {"kernel": "dd_valu (software FP64x2 on FP64 VALU)",
                                "ms": round(vms, 3), "value": round(flops_eff / (vms * 1e-3) / 1e9, 2),
                                "unit": "GFLOP/s", "cascade_speedup": round(vms / ms_per_step, 3)}
        Vs = (Vh.T[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy(),
              Vl.T[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy())
        del Vh, Vl

    if not args.no_comparator:
        # the paper states the cascade's cost as a multiple of DGEMM time on
        # the same machine (Sec. 5.1): time the vendor FP64 GEMM at this shape
        log("vendor DGEMM (torch.matmul, float64) at the same shape")
        X, Y = Ah.T, Bh.T                       # row-major views: Y @ X = (A B)^T
        Z = torch.empty((n, m), dtype=torch.float64, device="cuda")
        for _ in range(2):
            torch.matmul(Y, X, out=Z)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        ev0.record(stream)
        for _ in range(reps):
            torch.matmul(Y, X, out=Z)
        ev1.record(stream)
        torch.cuda.synchronize()
        gms = ev0.elapsed_time(ev1) / reps
        result["dgemm"] = {"library": "torch.matmul float64 (vendor BLAS)", "ms": round(gms, 3),
                           "tflops": round(2.0 * m * n * k / (gms * 1e-3) / 1e12, 2),
                           "cascade_time_over_dgemm": round(ms_per_step / gms, 2)}
        del Z

    if not args.no_comparator:
        # the paper's simple form: ten vendor DGEMMs per rank-kc update into
        # explicit bins, then a combine pass (same split and epilogue)
        log("unfused form: ten library DGEMMs per rank-kc update")
        Uh, Ul = C0h.clone(), C0l.clone()
        uopts = {"algo": dg.DD_ALGO_SIMPLE_UNFUSED}
        dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Uh, Ul, m, opts=uopts, stream=stream))
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Uh, Ul, m, opts=uopts, stream=stream))
        ev1.record(stream)
        torch.cuda.synchronize()
        ums = ev0.elapsed_time(ev1)
        result["simple_unfused"] = {"kernel": "split + 10 rocBLAS DGEMMs and a combine per rank-kc block",
                                    "ms": round(ums, 3), "value": round(flops_eff / (ums * 1e-3) / 1e9, 2),
                                    "unit": "GFLOP/s", "fused_speedup": round(ums / ms_per_step, 3)}
        del Uh, Ul

    # Sigma and T per rank-kc panel: the same product kernel with a per-block
    # scale in its combine; timed once at the headline shape
    Ph, Pl = C0h.clone(), C0l.clone()
    popts = {"scaling": dg.DD_SCALING_PANEL}
    dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ph, Pl, m, opts=popts, stream=stream))
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ph, Pl, m, opts=popts, stream=stream))
    ev1.record(stream)
    torch.cuda.synchronize()
    result["panel_scaling"] = {"ms": round(ev0.elapsed_time(ev1), 3),
                               "value": round(flops_eff / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 2),
                               "unit": "GFLOP/s"}
    del Ph, Pl
    # power-of-two diagonal balancing: two more reductions in the split
    Ph, Pl = C0h.clone(), C0l.clone()
    bopts = {"scaling": dg.DD_SCALING_BALANCE}
    dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ph, Pl, m, opts=bopts, stream=stream))
    torch.cuda.synchronize()
    ev0.record(stream)
    dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ph, Pl, m, opts=bopts, stream=stream))
    ev1.record(stream)
    torch.cuda.synchronize()
    result["balancing"] = {"ms": round(ev0.elapsed_time(ev1), 3),
                           "value": round(flops_eff / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 2),
                           "unit": "GFLOP/s"}
    del Ph, Pl

    # the split done while operands are staged (no digit planes in memory):
    # the same products and bits, the split repeated by every workgroup
    Ph, Pl = C0h.clone(), C0l.clone()
    oopts = {"algo": dg.DD_ALGO_CASCADE_ON_LOAD}
    dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ph, Pl, m, opts=oopts, stream=stream))
    torch.cuda.synchronize()
    Ph.copy_(C0h)
    Pl.copy_(C0l)
    ev0.record(stream)
    dg.check(dg.dd_gemm_ex(0, 0, m, n, k, Ah, Al, m, Bh, Bl, k, Ph, Pl, m, opts=oopts, stream=stream))
    ev1.record(stream)
    torch.cuda.synchronize()
    oms = ev0.elapsed_time(ev1)
    Ch2, Cl2 = C0h.clone(), C0l.clone()
    step_into = (Ch2, Cl2)
    dg.check(dg.dd_gemm(m, n, k, Ah, Al, m, Bh, Bl, k, step_into[0], step_into[1], m, stream), "dd_gemm")
    torch.cuda.synchronize()
    result["split_on_load"] = {
        "ms": round(oms, 3), "value": round(flops_eff / (oms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
        "time_over_packed_cascade": round(oms / ms_per_step, 4),
        "workspace_bytes": dg.dd_gemm_workspace_size(0, 0, m, n, k, oopts),
        "packed_workspace_bytes": dg.dd_gemm_workspace_size(0, 0, m, n, k),
        "bitwise_equal_to_packed_cascade": bool(torch.equal(Ph, Ch2) and torch.equal(Pl, Cl2))}
    del Ph, Pl, Ch2, Cl2

    if not args.no_cpu_baseline:
        from oracle.ref import dd_gemm_ref_entries  # CPU baseline leg only
        A, B, C = P["A"], P["B"], P["C"]
        probe = 2048
        t = time.perf_counter()
        dd_gemm_ref_entries(A, B, C, I[:probe], J[:probe])
        dt = time.perf_counter() - t
        S = int(min(len(I), max(probe, probe * args.oracle_seconds / max(dt, 1e-3))))
        log(f"oracle on {S} sampled entries (~{args.oracle_seconds:.0f} s)")
        t = time.perf_counter()
        Rh, Rl, used = dd_gemm_ref_entries(A, B, C, I[:S], J[:S])
        dt = time.perf_counter() - t
        result["cpu_baseline"] = {
            "value": round(2.0 * k * S / dt / 1e9, 4), "unit": "GFLOP/s", "cores": int(used),
            "kind": "oracle",
            "sample": f"{S} seeded output entries (i, j) of the same {m}x{n}x{k} problem, each a full "
                      f"length-{k} FP64x2 dot product plus C; {dt:.1f} s wall",
            "projected_full_s": round(dt * (m * n) / S, 1),
            "cpu_model": cpu_model(), "host_threads_available": os.cpu_count()}
        log("oracle on one host core at 1024")
        result["cpu_baseline"]["single_thread"] = oracle_single_thread_rate()
        diff = np.abs((Gh[:S] - Rh) + (Gl[:S] - Rl))
        denom = np.abs(Rh)
        nz = denom > 0
        rel = diff[nz] / denom[nz]
        log("tolerance scale |A||B| on every sampled entry")
        normed = diff / abs_ab_entries(A[0], B[0], I[:S], J[:S])
        result["accuracy"] = {
            "sampled_entries": S, "max_rel_err": float(np.max(rel)), "median_rel_err": float(np.median(rel)),
            "excluded_zero": int(np.sum(~nz)),
            "tolerance_checked_entries": int(len(normed)),
            "max_err_over_absAabsB": float(np.max(normed)),
            "median_err_over_absAabsB": float(np.median(normed)),
            "tolerance_over_absAabsB": 64 * k * 2.0 ** -104,
            "within_tolerance": bool(np.all(normed <= 64 * k * 2.0 ** -104))}
        if "comparator" in result:
            result["comparator"]["bitwise_equal_to_oracle_on_sample"] = bool(
                np.array_equal(Vs[0][:S], Rh) and np.array_equal(Vs[1][:S], Rl))
            vdiff = np.abs((Vs[0][:S] - Rh) + (Vs[1][:S] - Rl))
            result["comparator"]["max_rel_err"] = float(np.max(vdiff[nz] / denom[nz]))
    if not args.no_extras:
        log("batched: 512 uneven problems")
        result["batched"] = bench_batched(torch, dg, stream)
        log("differentiation chain")
        result["autograd"] = bench_autograd(torch)
        del Ah, Al, Bh, Bl, Ch, Cl, C0h, C0l, dev
        torch.cuda.empty_cache()
        result["sizes"] = bench_sizes(torch, dg, stream, cpu=not args.no_cpu_baseline)
        log("slices variant at 4096^3")
        sres, samples, IJ = bench_slices(torch, dg, stream)
        if not args.no_cpu_baseline:
            log("slices accuracy against the oracles (sampled entries)")
            slices_accuracy(sres, samples, IJ)
        result["slices"] = sres
        log("FP64x3 at 4096^3")
        result["fp64x3"] = bench_td(torch, dg, stream)
        if not args.no_cpu_baseline:
            td_accuracy(torch, dg, result["fp64x3"])
        result["fp64x3"].pop("_samples", None)
        if not args.no_cpu_baseline:
            log("accuracy workloads at n=240 against the exact product")
            result["accuracy_workloads"] = accuracy_workloads(torch, dg)
            log("panel scaling against global scaling on panel-scaled inputs")
            result["panel_scaling"].update(panel_scaling(torch, dg))
            log("balancing against global scaling on skewed inputs")
            result["balancing"].update(balancing(torch, dg))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
