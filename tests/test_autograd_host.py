"""CPU checks of how gradients of FP64x2 tensors are accumulated (host logic).

Gradients of the DD autograd functions are ``DDGrad`` tensors; torch's
autograd adds the gradients of a tensor used more than once (and a leaf's
gradients over several backward passes) with ``aten.add`` / ``aten.add_``,
which ``DDGrad`` turns into the FP64x2 addition.  Here the device addition
is replaced by the oracle's on the host, so the routing can be checked
without a GPU: plane-by-plane addition would lose the 2^-60 below.
"""
import numpy as np
import pytest
import torch

from oracle.ref import dd_add_ref
from paper_2303_04353_amd import autograd as ag

calls = []


@pytest.fixture(autouse=True)
def host_addition(monkeypatch):
    def add(z, x, y):
        z, x, y = ag.plain(z), ag.plain(x), ag.plain(y)
        h, l = dd_add_ref((x[0].numpy(), x[1].numpy()), (y[0].numpy(), y[1].numpy()))
        z[0].copy_(torch.from_numpy(h))
        z[1].copy_(torch.from_numpy(l))
        calls.append(z.shape)
        return z
    calls.clear()
    monkeypatch.setattr(ag, "dd_add_", add)


class Use(torch.autograd.Function):
    """y = x; the backward hands x the DD gradient given at forward time."""

    @staticmethod
    def forward(ctx, x, g):
        ctx.g = g
        return x.clone()

    @staticmethod
    def backward(ctx, dy):
        return ag.DDGrad(ctx.g.clone()), None


class Join(torch.autograd.Function):
    """A scalar from any number of inputs; backward sends zeros."""

    @staticmethod
    def forward(ctx, *xs):
        ctx.shapes = [x.shape for x in xs]
        return torch.zeros(2, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        return tuple(torch.zeros(s, dtype=torch.float64) for s in ctx.shapes)


def dd(h, l):
    return torch.tensor([h, l], dtype=torch.float64).reshape(2, 1)


def value(t):
    t = ag.plain(t)
    return (float(t[0, 0]), float(t[1, 0]))


def test_leaf_used_twice_gets_the_fp64x2_sum():
    x = torch.zeros(2, 1, dtype=torch.float64, requires_grad=True)
    y1 = Use.apply(x, dd(1.0, 0.0))
    y2 = Use.apply(x, dd(2.0 ** -60, 0.0))
    Join.apply(y1, y2).backward(torch.zeros(2, dtype=torch.float64))
    assert isinstance(x.grad, ag.DDGrad)
    assert value(x.grad) == (1.0, 2.0 ** -60)      # plane by plane: (1, 0)
    assert calls


def test_non_leaf_used_twice_and_three_times():
    x = torch.zeros(2, 1, dtype=torch.float64, requires_grad=True)
    h = Use.apply(x, dd(0.0, 0.0)) * 1.0               # a non-leaf DD tensor
    parts = [dd(1.0, 0.0), dd(2.0 ** -60, 0.0), dd(2.0 ** -61, 2.0 ** -120)]
    ys = [Use.apply(h, g) for g in parts]
    grads = []
    h.register_hook(lambda g: grads.append(g))
    Join.apply(*ys).backward(torch.zeros(2, dtype=torch.float64))
    got = value(grads[0])
    want = dd_add_ref(dd_add_ref(*[(p[0].numpy(), p[1].numpy()) for p in parts[:2]]),
                      (parts[2][0].numpy(), parts[2][1].numpy()))
    want2 = dd_add_ref((parts[0][0].numpy(), parts[0][1].numpy()),
                       dd_add_ref(*[(p[0].numpy(), p[1].numpy()) for p in parts[1:]]))
    assert got in ((float(want[0][0]), float(want[1][0])), (float(want2[0][0]), float(want2[1][0])))
    assert got[0] == 1.0 and got[1] == 2.0 ** -60 + 2.0 ** -61   # exact here in either order
    assert len(calls) >= 2


def test_leaf_accumulates_over_two_backward_passes():
    x = torch.zeros(2, 1, dtype=torch.float64, requires_grad=True)
    for g in (dd(1.0, 0.0), dd(2.0 ** -70, 0.0)):
        Join.apply(Use.apply(x, g)).backward(torch.zeros(2, dtype=torch.float64))
    assert value(x.grad) == (1.0, 2.0 ** -70)


def test_other_operations_see_the_planes():
    g = ag.DDGrad(torch.tensor([[3.0], [2.0 ** -60]], dtype=torch.float64))
    assert isinstance(g.detach(), ag.DDGrad)
    assert not isinstance(g * 2, ag.DDGrad)
    assert float((g * 2)[0, 0]) == 6.0
    assert np.array_equal(ag.plain(g).numpy(), np.array([[3.0], [2.0 ** -60]]))
    # an addition with a scale factor is not a DD sum: it runs plane by plane
    r = torch.add(g, g, alpha=2)
    assert not isinstance(r, ag.DDGrad) and float(r[0, 0]) == 9.0
    assert not calls
