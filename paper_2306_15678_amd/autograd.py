"""Differentiable march: a torch.autograd.Function over the library's
forward record and exact discrete adjoint.

``march(u0, theta, prop, n_steps)`` returns U_N (complex128, SI) of the
single beam of ``prop``; its backward seeds the library with torch's
cotangent (dL/dRe U_N + i dL/dIm U_N, torch's convention for a real loss)
and runs the hand-written adjoint (checkpoint recompute included), giving
dL/dU0 and dL/dtheta.  The context is stateful: do not run another march on
the same ``Propagator`` between this forward and its backward.

``lens(u_in, params, prop, i, template)`` applies the effective lens with
differentiable parameters; its backward is the library's vector-Jacobian
product, so march -> lens -> march chains (one context per march)
differentiate end to end.
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


def lens_params_vector(lens) -> list:
    """The differentiable lens parameters in the library's gradient order:
    c1, c2, then (amplitude, frequency, phase) of each real segment, then of
    each imaginary one."""
    v = [lens.c1, lens.c2]
    for j in range(lens.n_re):
        v += [lens.re[j][1], lens.re[j][2], lens.re[j][3]]
    for j in range(lens.n_im):
        v += [lens.im[j][1], lens.im[j][2], lens.im[j][3]]
    return v


def _lens_with(template, params: list):
    """A copy of ``template`` (its l_dif, w_l, segment ends and counts) with
    the differentiable parameters replaced by ``params``."""
    from .march import make_lens
    k = 2
    re, im = [], []
    for j in range(template.n_re):
        re.append((template.re[j][0], *params[k:k + 3]))
        k += 3
    for j in range(template.n_im):
        im.append((template.im[j][0], *params[k:k + 3]))
        k += 3
    return make_lens(template.l_dif, template.w_l, params[0], params[1], re, im)


class _Lens(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_in: torch.Tensor, params: torch.Tensor, prop: Propagator, i: int,
                template):
        lens = _lens_with(template, params.detach().to(torch.float64).cpu().tolist())
        u = u_in.detach().to(torch.complex128).contiguous()
        prop.set_field(i, u)
        prop.apply_lens(i, lens)
        out = prop.field(i, device=True)
        ctx.save_for_backward(u)
        ctx.prop, ctx.i, ctx.lens = prop, i, lens
        ctx.params_meta = (params.dtype, params.device)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (u,) = ctx.saved_tensors
        g_in, grad = ctx.prop.lens_vjp(ctx.i, ctx.lens, u, grad_out.detach())
        dt, dev = ctx.params_meta
        return g_in, torch.tensor(grad, dtype=dt, device=dev), None, None, None


def lens(u_in: torch.Tensor, params: torch.Tensor, prop: Propagator, i: int, template):
    """The effective lens applied to u_in (complex128 SI, instance i's grid)
    with the differentiable parameters ``params`` (order of
    ``lens_params_vector``) and the rest of ``template``; the context's
    field i is overwritten, its recorded march ended.  Differentiable in
    u_in and params through the library's vector-Jacobian product."""
    return _Lens.apply(u_in, params, prop, i, template)
