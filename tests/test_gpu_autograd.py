"""GPU checks of the differentiated chain L = sum((W2 (W1 X)) o G).

* forward, and every gradient of the hand-written cascaded backward, against
  the CPU reference built from FP64x2 oracle GEMMs (full matrices at a small
  size, sampled entries at W 2048 x 2048, X and G 2048 x 512);
* against FP64x2 central finite differences on 64 entries.  L is linear in
  every entry, so the central difference has no truncation error for any
  step; its rounding error is bounded from the error of L.
* dd_dot and dd_scal against the oracle.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle.ref import dd_gemm_ref
from paper_2303_04353_amd import autograd as ag
from paper_2303_04353_amd.inputs import make_pair
from tests.gpuhelp import log

pytestmark = pytest.mark.gpu
U = 2.0 ** -104


def dd_t(pair):
    return ag.dd_from_pair(np.ascontiguousarray(pair[0]), np.ascontiguousarray(pair[1])).cuda()


def np_pair(t):
    a = t.detach().cpu().numpy()
    return a[0], a[1]


def dd_val(h, l):
    return Fraction(float(h)) + Fraction(float(l))


def ref_chain(W1, W2, X, G):
    H = dd_gemm_ref(W1, X)[:2]
    Y = dd_gemm_ref(W2, H)[:2]
    n = Y[0].size
    L = dd_gemm_ref((Y[0].reshape(1, n), Y[1].reshape(1, n)), (G[0].reshape(n, 1), G[1].reshape(n, 1)))[:2]
    dH = dd_gemm_ref(W2, G, transa=True)[:2]
    return {"H": H, "Y": Y, "L": (L[0][0, 0], L[1][0, 0]), "dW2": dd_gemm_ref(G, H, transb=True)[:2],
            "dH": dH, "dW1": dd_gemm_ref(dH, X, transb=True)[:2], "dX": dd_gemm_ref(W1, dH, transa=True)[:2]}


def abs_chain(W1, W2, X, G):
    a1, a2, ax, ag_ = (np.abs(M[0]) for M in (W1, W2, X, G))
    aH = a1 @ ax
    adH = a2.T @ ag_
    return {"dW2": ag_ @ aH.T, "dW1": adH @ ax.T, "dX": a1.T @ adH, "L": float(np.sum((a2 @ aH) * ag_))}


def diff(G, R):
    return np.abs((G[0] - R[0]) + (G[1] - R[1]))


def test_small_chain_full_against_oracle():
    n, b = 70, 50
    W1, W2 = make_pair((n, n), seed=1), make_pair((n, n), seed=2)
    X, G = make_pair((n, b), seed=3), make_pair((n, b), seed=4)
    tW1, tW2, tX, tG = (dd_t(M).requires_grad_() for M in (W1, W2, X, G))
    L = ag.chain_loss(tW1, tW2, tX, tG)
    L.backward(torch_ones())
    R = ref_chain(W1, W2, X, G)
    S = abs_chain(W1, W2, X, G)
    tol = lambda key: 3 * 64 * n * U * S[key]
    Lg = L.detach().cpu().numpy()
    assert abs(dd_val(*Lg) - dd_val(*R["L"])) <= Fraction(tol("L"))
    for key, t in (("dW1", tW1), ("dW2", tW2), ("dX", tX)):
        assert np.all(diff(np_pair(t.grad), R[key]) <= tol(key)), key
    assert np.all(diff(np_pair(tG.grad), np_pair(ag.matmul(dd_t(W2), ag.matmul(dd_t(W1), dd_t(X))))) == 0)


def torch_ones():
    import torch
    return torch.tensor([1.0, 0.0], dtype=torch.float64, device="cuda")


def test_dot_and_scal_against_oracle():
    import torch
    x = make_pair((1, 100003), seed=5)
    y = make_pair((100003, 1), seed=6)
    r = ag.dd_dot_raw(dd_t(x), dd_t((y[0].T, y[1].T)))
    R = dd_gemm_ref(x, y)[:2]
    bound = 4 * 100003 * U * float((np.abs(x[0]) @ np.abs(y[0]))[0, 0])
    assert abs(dd_val(*r.cpu().numpy()) - dd_val(R[0][0, 0], R[1][0, 0])) <= Fraction(bound)
    X = dd_t(make_pair((37, 11), seed=7))
    alpha = (3.0 * 2.0 ** -7, 2.0 ** -70)
    Y = ag.dd_scale(torch.tensor(alpha, dtype=torch.float64), X)
    Ra = dd_gemm_ref((np_pair(X)[0].reshape(-1, 1), np_pair(X)[1].reshape(-1, 1)),
                     (np.array([[alpha[0]]]), np.array([[alpha[1]]])))[:2]
    got = np_pair(Y)
    assert np.array_equal(got[0].reshape(-1, 1), Ra[0]) and np.array_equal(got[1].reshape(-1, 1), Ra[1])


def _perturbed(base, pair, idx, h):
    """A copy of the DD tensor ``base`` with entry idx moved by h (rounded to
    FP64x2), and the exact value of the moved entry."""
    v = dd_val(pair[0][idx], pair[1][idx]) + Fraction(h)
    nh = float(v)
    nl = float(v - Fraction(nh))
    t = base.clone()
    t[0][idx] = nh
    t[1][idx] = nl
    return t, dd_val(nh, nl)


@pytest.mark.parametrize("h", [2.0 ** -20, 1.0])
def test_config_size_gradients_and_finite_differences(h):
    import torch
    n, b = 2048, 512
    log(f"autograd chain W {n}x{n}, X {n}x{b}, h={h}")
    W1, W2 = make_pair((n, n), seed=11), make_pair((n, n), seed=12)
    X, G = make_pair((n, b), seed=13), make_pair((n, b), seed=14)
    tW1, tW2, tX, tG = (dd_t(M).requires_grad_() for M in (W1, W2, X, G))
    L = ag.chain_loss(tW1, tW2, tX, tG)
    L.backward(torch_ones())
    torch.cuda.synchronize()
    grads = {"W1": np_pair(tW1.grad), "W2": np_pair(tW2.grad), "X": np_pair(tX.grad)}
    S = abs_chain(W1, W2, X, G)
    errL = 3 * 64 * n * U * S["L"]
    rng = np.random.default_rng(2303)
    picks = ([("W1", (int(i), int(j))) for i, j in rng.integers(0, n, size=(22, 2))]
             + [("W2", (int(i), int(j))) for i, j in rng.integers(0, n, size=(21, 2))]
             + [("X", (int(i), int(j))) for i, j in zip(rng.integers(0, n, 21), rng.integers(0, b, 21))])
    mats = {"W1": W1, "W2": W2, "X": X}
    base = {"W1": tW1.detach(), "W2": tW2.detach(), "X": tX.detach()}
    key_s = {"W1": "dW1", "W2": "dW2", "X": "dX"}
    worst = 0.0
    for name, idx in picks:
        Lpm = []
        steps = []
        for sgn in (+1, -1):
            pert, w = _perturbed(base[name], mats[name], idx, sgn * h)
            args = dict(base)
            args[name] = pert
            with torch.no_grad():
                Lv = ag.chain_loss(args["W1"], args["W2"], args["X"], tG.detach()).cpu().numpy()
            Lpm.append(dd_val(*Lv))
            steps.append(w)
        delta = steps[0] - steps[1]
        g_fd = (Lpm[0] - Lpm[1]) / delta
        g = dd_val(grads[name][0][idx], grads[name][1][idx])
        tol_g = 2 * 64 * n * U * S[key_s[name]][idx]
        bound = Fraction(2 * errL) / abs(delta) + Fraction(tol_g)
        err = abs(g_fd - g)
        worst = max(worst, float(err / bound))
        assert err <= bound, (name, idx, float(err), float(bound))
    log(f"finite differences: worst error / bound = {worst:.3e}")
    # sampled entries of every gradient against the CPU reference gradient
    for name, idx in picks[::8]:
        i, j = idx
        if name == "W1":      # dW1[i, j] = sum_p dH[i, p] X[j, p], dH = W2^T G
            dh = dd_gemm_ref((W2[0][:, i:i + 1].T, W2[1][:, i:i + 1].T), G)[:2]
            r = dd_gemm_ref(dh, (X[0][j:j + 1].T, X[1][j:j + 1].T))[:2]
        elif name == "W2":    # dW2[i, j] = sum_p G[i, p] H[j, p], H = W1 X
            hrow = dd_gemm_ref((W1[0][j:j + 1], W1[1][j:j + 1]), X)[:2]
            r = dd_gemm_ref((G[0][i:i + 1], G[1][i:i + 1]), (hrow[0].T, hrow[1].T))[:2]
        else:                 # dX[i, j] = sum_q W1[q, i] dH[q, j]
            dhc = dd_gemm_ref(W2, (G[0][:, j:j + 1], G[1][:, j:j + 1]), transa=True)[:2]
            r = dd_gemm_ref((W1[0][:, i:i + 1].T, W1[1][:, i:i + 1].T), dhc)[:2]
        g = dd_val(grads[name][0][idx], grads[name][1][idx])
        assert abs(g - dd_val(r[0][0, 0], r[1][0, 0])) <= Fraction(2 * 64 * n * U * S[key_s[name]][idx])


def test_dd_add_and_device_scalar_against_oracle():
    """dd_add equals the oracle's accurate FP64x2 addition bit for bit
    (heavy cancellation, strides, in place); dd_scal takes its scalar from
    device memory: a dot product computed on the device scales a vector with
    no host round trip, equal to the oracle's DD product."""
    import torch
    from oracle.ref import dd_add_ref
    from paper_2303_04353_amd import ddgemm as dg
    rng = np.random.default_rng(83)
    n = 100003
    xh = rng.uniform(-1, 1, n) * np.ldexp(1.0, rng.integers(-30, 30, n))
    xl = xh * rng.uniform(-1, 1, n) * 2.0 ** -53
    yh = -xh * (1 + rng.integers(-8, 9, n) * 2.0 ** -52)
    yh[::3] = rng.uniform(-1, 1, len(yh[::3]))
    yl = yh * rng.uniform(-1, 1, n) * 2.0 ** -53
    want = dd_add_ref((xh, xl), (yh, yl))
    d = [torch.from_numpy(v.copy()).cuda() for v in (xh, xl, yh, yl)]
    zh, zl = torch.empty_like(d[0]), torch.empty_like(d[0])
    dg.check(dg.dd_add(n, d[0], d[1], 1, d[2], d[3], 1, zh, zl, 1), "dd_add")
    torch.cuda.synchronize()
    assert np.array_equal(zh.cpu().numpy(), want[0]) and np.array_equal(zl.cpu().numpy(), want[1])
    # strided operands (every third entry of x, every second of y), result in place over y
    m = n // 3
    dg.check(dg.dd_add(m, d[0], d[1], 3, d[2], d[3], 2, d[2], d[3], 2), "dd_add strided")
    torch.cuda.synchronize()
    w2 = dd_add_ref((xh[::3][:m], xl[::3][:m]), (yh[::2][:m], yl[::2][:m]))
    assert np.array_equal(d[2].cpu().numpy()[::2][:m], w2[0]) and np.array_equal(d[3].cpu().numpy()[::2][:m], w2[1])
    assert np.array_equal(d[2].cpu().numpy()[1::2], yh[1::2])        # untouched between the strides
    # the scalar of dd_scal comes from a device computation
    x = make_pair((1, 4097), seed=15)
    y = make_pair((4097, 1), seed=16)
    r = ag.dd_dot_raw(dd_t(x), dd_t((y[0].T, y[1].T)))          # on the device
    X = dd_t(make_pair((33, 7), seed=17))
    Y = ag.dd_scale(r, X)
    alpha = r.cpu().numpy()
    Ra = dd_gemm_ref((np_pair(X)[0].reshape(-1, 1), np_pair(X)[1].reshape(-1, 1)),
                     (np.array([[alpha[0]]]), np.array([[alpha[1]]])))[:2]
    got = np_pair(Y)
    assert np.array_equal(got[0].reshape(-1, 1), Ra[0]) and np.array_equal(got[1].reshape(-1, 1), Ra[1])


def reuse_ref(W, X, G):
    """Oracle gradients of L = sum((W (W X)) o G): dW = G H^T + W^T G X^T
    (the two uses of W, added in FP64x2), dX = W^T (W^T G)."""
    from oracle.ref import dd_add_ref
    H = dd_gemm_ref(W, X)[:2]
    Y = dd_gemm_ref(W, H)[:2]
    n = Y[0].size
    L = dd_gemm_ref((Y[0].reshape(1, n), Y[1].reshape(1, n)), (G[0].reshape(n, 1), G[1].reshape(n, 1)))[:2]
    dH = dd_gemm_ref(W, G, transa=True)[:2]
    dW = dd_add_ref(dd_gemm_ref(G, H, transb=True)[:2], dd_gemm_ref(dH, X, transb=True)[:2])
    return {"L": (L[0][0, 0], L[1][0, 0]), "dW": dW, "dX": dd_gemm_ref(W, dH, transa=True)[:2]}


def reuse_abs(W, X, G):
    aw, ax, ag_ = (np.abs(M[0]) for M in (W, X, G))
    aH = aw @ ax
    adH = aw.T @ ag_
    return {"dW": ag_ @ aH.T + adH @ ax.T, "dX": aw.T @ adH, "L": float(np.sum((aw @ aH) * ag_)),
            "quad": ag_ @ ax.T}


def reuse_loss(W, X, G):
    return ag.dot(ag.matmul(W, ag.matmul(W, X)), G)


def test_reused_weight_small_full_against_oracle():
    """A DD tensor used twice: L = sum((W (W X)) o G).  The gradient of W is
    the FP64x2 sum of the two uses' gradients (a DDGrad accumulation), held
    to the oracle's within four times the GEMM tolerance of each term;
    plane-by-plane addition would miss it by about 2^-53 |dW|."""
    n, b = 96, 40
    W, X, G = make_pair((n, n), seed=21), make_pair((n, b), seed=22), make_pair((n, b), seed=23)
    tW, tX, tG = (dd_t(M).requires_grad_() for M in (W, X, G))
    L = reuse_loss(tW, tX, tG)
    L.backward(torch_ones())
    assert isinstance(tW.grad, ag.DDGrad)
    R = reuse_ref(W, X, G)
    S = reuse_abs(W, X, G)
    assert abs(dd_val(*L.detach().cpu().numpy()) - dd_val(*R["L"])) <= Fraction(3 * 64 * n * U * S["L"])
    for key, t in (("dW", tW), ("dX", tX)):
        tol = 4 * 64 * n * U * S[key] + 2.0 ** -100 * np.abs(R[key][0])
        assert np.all(diff(np_pair(t.grad), R[key]) <= tol), key
    # the same gradient formed plane by plane misses the tolerance
    import torch
    g1 = ag.gemm(dd_t(G), ag.gemm(dd_t(W), dd_t(X)), transY=True)
    g2 = ag.gemm(ag.gemm(dd_t(W), dd_t(G), transX=True), dd_t(X), transY=True)
    planes = np_pair(g1 + g2)
    assert not np.all(diff(planes, R["dW"]) <= 4 * 64 * n * U * S["dW"])
    torch.cuda.synchronize()


def test_reused_weight_config_size_finite_differences():
    """L = sum((W (W X)) o G) with W 2048^2, X, G 2048 x 512: gradients of 64
    entries (43 of W, 21 of X) against FP64x2 central differences.  L is
    linear in X and in every off-diagonal entry of W, and quadratic in a
    diagonal entry W_aa with coefficient (G X^T)_aa, so the difference over
    the steps actually taken is exact up to (G X^T)_aa (w+ + w- - 2 w)."""
    import torch
    n, b, h = 2048, 512, 2.0 ** -20
    W, X, G = make_pair((n, n), seed=31), make_pair((n, b), seed=32), make_pair((n, b), seed=33)
    log(f"reused weight chain W {n}x{n}, X {n}x{b}")
    tW, tX, tG = (dd_t(M).requires_grad_() for M in (W, X, G))
    reuse_loss(tW, tX, tG).backward(torch_ones())
    torch.cuda.synchronize()
    grads = {"W": np_pair(tW.grad), "X": np_pair(tX.grad)}
    S = reuse_abs(W, X, G)
    errL = 3 * 64 * n * U * S["L"]
    rng = np.random.default_rng(2304)
    picks = ([("W", (int(i), int(j))) for i, j in rng.integers(0, n, size=(40, 2))]
             + [("W", (int(i), int(i))) for i in rng.integers(0, n, 3)]
             + [("X", (int(i), int(j))) for i, j in zip(rng.integers(0, n, 21), rng.integers(0, b, 21))])
    mats, base = {"W": W, "X": X}, {"W": tW.detach(), "X": tX.detach()}
    worst = 0.0
    for name, idx in picks:
        Lpm, steps = [], []
        for sgn in (+1, -1):
            pert, w = _perturbed(base[name], mats[name], idx, sgn * h)
            args = dict(base)
            args[name] = pert
            with torch.no_grad():
                Lpm.append(dd_val(*reuse_loss(args["W"], args["X"], tG.detach()).cpu().numpy()))
            steps.append(w)
        delta = steps[0] - steps[1]
        g_fd = (Lpm[0] - Lpm[1]) / delta
        g = dd_val(grads[name][0][idx], grads[name][1][idx])
        key = "d" + name
        tol_g = 2 * 64 * n * U * S[key][idx] + 3 * U * abs(float(g))
        quad = 0
        if name == "W" and idx[0] == idx[1]:
            w0 = dd_val(mats["W"][0][idx], mats["W"][1][idx])
            quad = Fraction(float(S["quad"][idx])) * abs(steps[0] + steps[1] - 2 * w0)
        bound = Fraction(2 * errL) / abs(delta) + Fraction(tol_g) + quad
        err = abs(g_fd - g)
        worst = max(worst, float(err / bound))
        assert err <= bound, (name, idx, float(err), float(bound))
    log(f"reused weight, finite differences: worst error / bound = {worst:.3e}")
