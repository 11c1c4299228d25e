"""FP64x2 tensors and differentiation through the cascaded GEMM.

An FP64x2 ("DD") tensor here is a torch float64 tensor of shape
``(2, *shape)`` on the GPU: plane 0 holds the high words, plane 1 the low
words, each plane row-major and contiguous.  The value of an entry is
``t[0][idx] + t[1][idx]`` taken exactly.

* :func:`matmul` -- ``A @ B`` for DD matrices through ``dd_gemm_ex``; its
  backward is itself cascaded: ``dA = dC B^T`` and ``dB = A^T dC`` (two more
  cascaded GEMMs with transposed operands).
* :func:`dot` -- ``sum(Y * G)`` as a DD scalar ``(2,)``; backward
  ``dY = g G``, ``dG = g Y`` (``dd_scal``).

torch's autograd adds the gradients of a tensor that is used more than once
plane by plane, which is not an FP64x2 addition; the functions here are meant
for chains in which each DD tensor is used once (as in the benchmarked
chain L = sum((W2 (W1 X)) o G)).
"""
from __future__ import annotations

import torch

from . import ddgemm as dg


def dd_zeros(*shape, device="cuda"):
    return torch.zeros((2,) + tuple(shape), dtype=torch.float64, device=device)


def dd_from_pair(hi, lo):
    """Stack two float64 tensors (or numpy arrays) of equal shape into a DD tensor."""
    hi = torch.as_tensor(hi, dtype=torch.float64)
    lo = torch.as_tensor(lo, dtype=torch.float64)
    return torch.stack([hi, lo]).contiguous()


def _check(t, name, ndim):
    if t.dtype != torch.float64 or t.dim() != ndim + 1 or t.shape[0] != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 DD tensor of shape (2, ...) with {ndim} dims")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")


def gemm(X, Y, *, transX=False, transY=False, out=None, kc=0):
    """``out += op(X) @ op(Y)`` (``out`` zero if not given) for row-major DD matrices."""
    _check(X, "X", 2)
    _check(Y, "Y", 2)
    M = X.shape[2] if transX else X.shape[1]
    K = X.shape[1] if transX else X.shape[2]
    KY = Y.shape[2] if transY else Y.shape[1]
    N = Y.shape[1] if transY else Y.shape[2]
    if K != KY:
        raise ValueError(f"inner dimensions differ: {K} vs {KY}")
    if out is None:
        out = dd_zeros(M, N, device=X.device)
    else:
        _check(out, "out", 2)
        if tuple(out.shape[1:]) != (M, N):
            raise ValueError("out has the wrong shape")
    # A row-major r x c matrix is the column-major c x r matrix with ld = c:
    # out^T = op(Y)^T op(X)^T in column-major terms.
    st = dg.dd_gemm_ex(int(transY), int(transX), N, M, K,
                       Y[0], Y[1], max(1, Y.shape[2]), X[0], X[1], max(1, X.shape[2]),
                       out[0], out[1], max(1, N), opts={"kc": kc})
    dg.check(st, "dd_gemm_ex")
    return out


def dd_dot_raw(Y, G):
    """``sum(Y * G)`` as a DD scalar tensor ``(2,)``."""
    n = Y[0].numel()
    if G[0].numel() != n:
        raise ValueError("dot of tensors of different sizes")
    res = torch.empty(2, dtype=torch.float64, device=Y.device)
    dg.check(dg.dd_dot(n, Y[0], Y[1], 1, G[0], G[1], 1, res), "dd_dot")
    return res


def dd_scale(alpha, X):
    """``alpha * X`` for a DD scalar ``alpha`` (a ``(2,)`` tensor or a (hi, lo) pair)."""
    if torch.is_tensor(alpha):
        ah, al = (float(v) for v in alpha.detach().cpu().tolist())
    else:
        ah, al = float(alpha[0]), float(alpha[1])
    Y = torch.empty_like(X)
    n = X[0].numel()
    dg.check(dg.dd_scal(n, ah, al, X[0], X[1], 1, Y[0], Y[1], 1), "dd_scal")
    return Y


class DDMatmul(torch.autograd.Function):
    """C = A @ B for DD matrices ``(2, M, K)``, ``(2, K, N)`` -> ``(2, M, N)``."""

    @staticmethod
    def forward(ctx, A, B):
        ctx.save_for_backward(A, B)
        return gemm(A, B)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dC = dC.contiguous()
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = gemm(dC, B, transY=True)          # dA = dC B^T
        if ctx.needs_input_grad[1]:
            dB = gemm(A, dC, transX=True)          # dB = A^T dC
        return dA, dB


class DDDot(torch.autograd.Function):
    """L = sum(Y * G) as a DD scalar ``(2,)``."""

    @staticmethod
    def forward(ctx, Y, G):
        ctx.save_for_backward(Y, G)
        return dd_dot_raw(Y, G)

    @staticmethod
    def backward(ctx, gL):
        Y, G = ctx.saved_tensors
        dY = dG = None
        if ctx.needs_input_grad[0]:
            dY = dd_scale(gL, G)
        if ctx.needs_input_grad[1]:
            dG = dd_scale(gL, Y)
        return dY, dG


def matmul(A, B):
    return DDMatmul.apply(A, B)


def dot(Y, G):
    return DDDot.apply(Y, G)


def chain_loss(W1, W2, X, G):
    """L = sum((W2 (W1 X)) o G), the differentiated chain of the benchmark."""
    return dot(matmul(W2, matmul(W1, X)), G)
