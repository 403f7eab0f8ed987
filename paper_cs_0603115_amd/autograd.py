"""torch.autograd.Function wrappers with hand-written float-float backward
kernels.

Gradient convention: a float-float tensor has shape (2, ...) and its value
is plane 0 + plane 1.  The gradient autograd carries for it has the same
shape and holds, as a float-float number, dL/d(value) -- the derivative with
respect to the represented number (which is also the derivative with respect
to either plane).  The backward kernels read and write gradients in that
form.  A scalar float-float loss is seeded with the float-float one,
``loss.backward(torch.tensor([1.0, 0.0], device=...))``.

Ordinary torch operations on the planes follow the other convention: a loss
computed from the value, e.g. ``(w * (y[0] + y[1])).sum()``, sends each
plane its own partial derivative, and d/d(hi) = d/d(lo) = d/d(value), so
both planes carry the same number g.  A normalised float-float gradient
never has two equal planes except at zero (|lo| <= ulp(hi)/2), so the
backward functions read an element whose two planes are equal as the value
g itself, (g, g) -> (g, 0), and any other element as the float-float value
hi + lo.  (Selecting a plane is exact; no arithmetic is involved.)
"""
from __future__ import annotations

import torch

from . import (MATVEC_FAST, ff_dot_backward, ff_dot_batched_backward, ff_dot_ff_batched,
               ff_matvec, ff_matvec_backward)

__all__ = ["FFMatVec", "FFDot", "FFDotBatched", "ff_one"]


def _value_gradient(g: torch.Tensor) -> torch.Tensor:
    """The incoming gradient as a float-float value: elements whose two
    planes are equal (the per-plane derivative delivered by ordinary torch
    operations) keep plane 0 and get a zero low word."""
    g = g.contiguous()
    lo = torch.where(g[0] == g[1], torch.zeros_like(g[1]), g[1])
    return torch.stack((g[0], lo))


def ff_one(device="cuda") -> torch.Tensor:
    """The float-float number 1 (seed for a scalar loss)."""
    return torch.tensor([1.0, 0.0], dtype=torch.float32, device=device)


class FFMatVec(torch.autograd.Function):
    """y = A x (A: (2, M, N), x: (2, N), y: (2, M)); backward by
    ff_matvec_backward: dA = g x^T, dx = A^T g."""

    @staticmethod
    def forward(ctx, A, x, algo=MATVEC_FAST):
        ctx.save_for_backward(A, x)
        ctx.algo = algo
        return ff_matvec(A, x, algo=algo)

    @staticmethod
    def backward(ctx, gy):
        A, x = ctx.saved_tensors
        gy = _value_gradient(gy)
        dA, dx = ff_matvec_backward(A, x, gy, want_dA=ctx.needs_input_grad[0],
                                    want_dx=ctx.needs_input_grad[1], algo=ctx.algo)
        return dA, dx, None


class FFDot(torch.autograd.Function):
    """s = sum_i u_i v_i for float-float vectors u, v (2, n); s has shape (2,).
    Backward: du = g v, dv = g u (ff_dot_backward)."""

    @staticmethod
    def forward(ctx, u, v):
        ctx.save_for_backward(u, v)
        n = u.shape[1]
        offsets = torch.tensor([0, n], dtype=torch.int64, device=u.device)
        return ff_dot_ff_batched(u, v, offsets).reshape(2)

    @staticmethod
    def backward(ctx, gs):
        u, v = ctx.saved_tensors
        du, dv = ff_dot_backward(_value_gradient(gs), u, v, want_dx=ctx.needs_input_grad[0],
                                 want_dy=ctx.needs_input_grad[1])
        return du, dv


class FFDotBatched(torch.autograd.Function):
    """s_v = sum over [offsets[v], offsets[v+1]) of x_i y_i for float-float
    vectors x, y (2, total); s has shape (2, nvec).  Backward by
    ff_dot_batched_backward: dx_i = g_v y_i, dy_i = g_v x_i."""

    @staticmethod
    def forward(ctx, x, y, offsets):
        ctx.save_for_backward(x, y, offsets)
        return ff_dot_ff_batched(x, y, offsets)

    @staticmethod
    def backward(ctx, gs):
        x, y, offsets = ctx.saved_tensors
        dx, dy = ff_dot_batched_backward(_value_gradient(gs), x, y, offsets,
                                         want_dx=ctx.needs_input_grad[0],
                                         want_dy=ctx.needs_input_grad[1])
        return dx, dy, None
