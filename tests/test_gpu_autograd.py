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
