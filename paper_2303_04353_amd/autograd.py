"""FP64x2 tensors and differentiation through the cascaded GEMM.

An FP64x2 ("DD") tensor here is a torch float64 tensor of shape
``(2, *shape)`` on the GPU: plane 0 holds the high words, plane 1 the low
words, each plane row-major and contiguous.  The value of an entry is
``t[0][idx] + t[1][idx]`` taken exactly.

* :func:`matmul` -- ``A @ B`` for DD matrices through ``dd_gemm_ex``; its
  backward is itself cascaded: ``dA = dC B^T`` and ``dB = A^T dC`` (two more
  cascaded GEMMs with transposed operands).
* :func:`dot` -- ``sum(Y * G)`` as a DD scalar ``(2,)``; backward
  ``dY = g G``, ``dG = g Y`` (``dd_scal``, with the scalar g read on the
  device: no host synchronisation).

Gradients are returned as :class:`DDGrad` tensors.  When a DD tensor feeds
several operations, torch's autograd adds the gradients that reach it (and,
for a leaf, adds every backward pass into ``.grad``); for ``DDGrad`` those
additions run as the accurate FP64x2 addition (``dd_add``), not plane by
plane, so a reused tensor (``W (W X)``) gets an FP64x2 gradient.
"""
from __future__ import annotations

import torch
from torch.utils._pytree import tree_map

from . import ddgemm as dg

_aten = torch.ops.aten


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


def plain(t):
    """The plain DD tensor behind a :class:`DDGrad` (any other tensor as is)."""
    return t._dd if isinstance(t, DDGrad) else t


def dd_add_(z, x, y):
    """``z = x + y`` for DD tensors of one shape, entry by entry with the
    accurate FP64x2 addition (``dd_add``); z may be x or y.  Returns z."""
    z, x, y = plain(z), plain(x).contiguous(), plain(y).contiguous()
    if not (z.shape == x.shape == y.shape) or z.shape[0] != 2 or not z.is_contiguous():
        raise ValueError("dd_add_: DD tensors (2, ...) of one shape, z contiguous")
    if x.dtype != torch.float64 or y.dtype != torch.float64 or z.dtype != torch.float64:
        raise ValueError("dd_add_: float64 DD tensors")
    n = z[0].numel()
    dg.check(dg.dd_add(n, x[0], x[1], 1, y[0], y[1], 1, z[0], z[1], 1), "dd_add")
    return z


class DDGrad(torch.Tensor):
    """A gradient of a DD tensor, a wrapper around a plain ``(2, *shape)``
    float64 tensor.  ``a + b`` and ``a += b`` between DD gradients (or a DD
    gradient and a plain DD tensor, taken as hi and lo planes) are the
    accurate FP64x2 addition; every other operation works on the planes of
    the wrapped tensor and returns plain tensors."""

    @staticmethod
    def __new__(cls, data):
        data = plain(data)
        r = torch.Tensor._make_wrapper_subclass(cls, data.shape, dtype=data.dtype, device=data.device,
                                                strides=data.stride(), requires_grad=False)
        r._dd = data
        return r

    def __repr__(self):
        return f"DDGrad({self._dd!r})"

    @classmethod
    def __torch_dispatch__(cls, func, types, args=(), kwargs=None):
        kwargs = kwargs or {}
        if func in (_aten.add.Tensor, _aten.add_.Tensor) and kwargs.get("alpha", 1) == 1 and len(args) == 2:
            x, y = args
            if torch.is_tensor(x) and torch.is_tensor(y) and x.shape == y.shape and x.dim() >= 1 \
                    and x.shape[0] == 2 and x.dtype == y.dtype == torch.float64:
                if func is _aten.add_.Tensor:
                    target = plain(x)
                    if target.is_contiguous():
                        dd_add_(target, x, y)
                        return x
                out = torch.empty_like(plain(x), memory_format=torch.contiguous_format)
                dd_add_(out, x, y)
                if func is _aten.add_.Tensor:
                    plain(x).copy_(out)
                    return x
                return DDGrad(out)
        if func in (_aten.detach.default, _aten.alias.default):
            return DDGrad(func(plain(args[0])))
        return func(*tree_map(plain, args), **tree_map(plain, kwargs))


def gemm(X, Y, *, transX=False, transY=False, out=None, kc=0):
    """``out += op(X) @ op(Y)`` (``out`` zero if not given) for row-major DD matrices."""
    X, Y = plain(X), plain(Y)
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
    Y, G = plain(Y), plain(G)
    n = Y[0].numel()
    if G[0].numel() != n:
        raise ValueError("dot of tensors of different sizes")
    res = torch.empty(2, dtype=torch.float64, device=Y.device)
    dg.check(dg.dd_dot(n, Y[0], Y[1], 1, G[0], G[1], 1, res), "dd_dot")
    return res


def dd_scale(alpha, X):
    """``alpha * X`` for a DD scalar ``alpha``: a ``(2,)`` tensor, read on
    the device (no host synchronisation), or a host ``(hi, lo)`` pair."""
    X = plain(X)
    if torch.is_tensor(alpha):
        a = plain(alpha).detach()
        if a.numel() != 2 or a.dtype != torch.float64:
            raise ValueError("alpha must hold two float64 words (hi, lo)")
        a = a.reshape(2).to(X.device).contiguous()
    else:
        a = torch.tensor([float(alpha[0]), float(alpha[1])], dtype=torch.float64, device=X.device)
    Y = torch.empty_like(X)
    n = X[0].numel()
    dg.check(dg.dd_scal(n, a, X[0], X[1], 1, Y[0], Y[1], 1), "dd_scal")
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
        dC = plain(dC).contiguous()
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = DDGrad(gemm(dC, B, transY=True))          # dA = dC B^T
        if ctx.needs_input_grad[1]:
            dB = DDGrad(gemm(A, dC, transX=True))          # dB = A^T dC
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
            dY = DDGrad(dd_scale(gL, G))
        if ctx.needs_input_grad[1]:
            dG = DDGrad(dd_scale(gL, Y))
        return dY, dG


def matmul(A, B):
    return DDMatmul.apply(A, B)


def dot(Y, G):
    return DDDot.apply(Y, G)


def chain_loss(W1, W2, X, G):
    """L = sum((W2 (W1 X)) o G), the differentiated chain of the benchmark."""
    return dot(matmul(W2, matmul(W1, X)), G)
