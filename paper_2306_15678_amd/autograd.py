"""Differentiable march: a torch.autograd.Function over the library's
forward record and exact discrete adjoint.

``march(u0, theta, prop, n_steps)`` returns U_N (complex128, SI) of the
single beam of ``prop``; its backward seeds the library with torch's
cotangent (dL/dRe U_N + i dL/dIm U_N, torch's convention for a real loss)
and runs the hand-written adjoint (checkpoint recompute included), giving
dL/dU0 and dL/dtheta.  The context is stateful: do not run another march on
the same ``Propagator`` between this forward and its backward.
"""
from __future__ import annotations

import torch

from .march import Propagator


class _March(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0: torch.Tensor, theta: torch.Tensor, prop: Propagator,
                n_steps: int):
        prop.set_field(0, u0.detach().to(torch.complex128).contiguous())
        prop.set_theta(0, theta.detach().to(torch.float64).cpu().tolist())
        prop.forward_record(n_steps)
        out = prop.field(0, device=True)
        ctx.prop = prop
        ctx.theta_meta = (theta.dtype, theta.device)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        p = ctx.prop
        p.set_cotangent(0, grad_out.detach().to(torch.complex128).contiguous())
        p.backward()
        g_u0 = p.grad_field(0, device=True)
        dt, dev = ctx.theta_meta
        g_th = torch.tensor(p.grad_theta(0), dtype=dt, device=dev)
        return g_u0, g_th, None, None


def march(u0: torch.Tensor, theta: torch.Tensor, prop: Propagator, n_steps: int) -> torch.Tensor:
    """U_N of the single beam of ``prop`` (created with max_steps >= n_steps)."""
    if prop.n_inst != 1:
        raise ValueError("march() drives single-beam contexts")
    return _March.apply(u0, theta, prop, n_steps)
