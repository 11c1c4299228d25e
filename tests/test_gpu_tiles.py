"""GPU checks of the output tile shapes of the cascade (64 x 64, 32 x 64,
64 x 32) and of the tile-shape tuner.

Every shape computes every entry with the same arithmetic (the same MFMA
instruction, inner order and combine), so results must be bit-identical
to the default shape: ragged and tiny shapes, transposes, per-panel
scaling with balancing, cancellation flags.  dd_tune records a shape per
problem, and use_tuned = 1 runs it.
"""
import numpy as np
import pytest

from paper_2303_04353_amd import ddgemm as dg
from paper_2303_04353_amd.inputs import make_problem
from tests.gpuhelp import down, log, up

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (33, 70, 257), (64, 64, 64), (96, 200, 300), (130, 33, 520), (200, 128, 40), (517, 300, 700)]


def _run(P, m, n, k, opts, transa=False, transb=False):
    import torch
    A = (up(P["A"][0]), up(P["A"][1]))
    B = (up(P["B"][0]), up(P["B"][1]))
    Ch, Cl = up(P["C"][0]), up(P["C"][1])
    o = dict(opts)
    fl = None
    if o.pop("flags", False):
        fl = torch.zeros(((m * n + 31) // 32,), dtype=torch.int32, device="cuda")
        o["flags_out"] = fl.data_ptr()
    st = dg.dd_gemm_ex(int(transa), int(transb), m, n, k, A[0], A[1], max(1, P["A"][0].shape[0]), B[0], B[1],
                       max(1, P["B"][0].shape[0]), Ch, Cl, m, opts=o)
    dg.check(st, "dd_gemm_ex")
    torch.cuda.synchronize()
    return down(Ch), down(Cl), (None if fl is None else fl.cpu().numpy())


@pytest.mark.parametrize("extra", [{}, {"kc": 64}, {"scaling": dg.DD_SCALING_PANEL | dg.DD_SCALING_BALANCE, "kc": 128},
                                   {"flags": True}], ids=["plain", "kc64", "panel+balance", "flags"])
def test_every_tile_shape_is_bit_identical(extra):
    for (m, n, k) in SHAPES:
        log(f"tiles {extra} {m}x{n}x{k}")
        P = make_problem(m, n, k, cfg=60, variant="scaled")
        ref = _run(P, m, n, k, dict(extra, tile=dg.DD_TILE_AUTO))
        for tile in (dg.DD_TILE_64x64, dg.DD_TILE_32x64, dg.DD_TILE_64x32):
            got = _run(P, m, n, k, dict(extra, tile=tile))
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (m, n, k, tile)
            if ref[2] is not None:
                assert np.array_equal(got[2], ref[2]), (m, n, k, tile)


def test_tile_shapes_with_transposes():
    m, n, k = 150, 90, 333
    P = make_problem(m, n, k, cfg=61)
    Q = {"A": tuple(np.asfortranarray(x.T) for x in P["A"]), "B": tuple(np.asfortranarray(x.T) for x in P["B"]),
         "C": P["C"]}
    ref = _run(P, m, n, k, {})
    for tile in (dg.DD_TILE_32x64, dg.DD_TILE_64x32):
        got = _run(Q, m, n, k, {"tile": tile}, transa=True, transb=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), tile


def test_tuner_records_and_use_tuned_runs_it(tmp_path, monkeypatch):
    monkeypatch.setenv("DDGEMM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ms, ns, ks = [512, 96, 0], [512, 1000, 5], [256, 300, 7]
    st, shapes = dg.dd_tune(ms, ns, ks, repeats=2)
    assert st == 0 and shapes[2] == 0 and all(s in (1, 2, 3) for s in shapes[:2])
    lines = [l.split() for l in open(tmp_path / "tune.txt").read().splitlines()]
    assert [l[0] for l in lines] == ["s", "s"]
    assert [int(l[6]) for l in lines] == shapes[:2]
    assert [(int(l[1]), int(l[2]), int(l[3]), int(l[4])) for l in lines] == [(512, 512, 256, 256), (96, 1000, 300, 256)]
    for (m, n, k) in zip(ms[:2], ns[:2], ks[:2]):
        P = make_problem(m, n, k, cfg=62)
        ref = _run(P, m, n, k, {})
        got = _run(P, m, n, k, {"use_tuned": 1})
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    log(f"tuned tile shapes: {shapes[:2]}")
