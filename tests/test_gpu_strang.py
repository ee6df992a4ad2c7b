"""Strang splitting on the GPU against the oracle's Strang march.

The library keeps V = L(dz/2) U between Strang steps (the Lie machinery with
each step's own screen applied on load), adds a half step when a field is
set and a backward half step when it is read.  Checked: FP64 fields and
per-step power against the oracle, the documented per-step peak (that of
L(dz/2) U), second-order convergence of the GPU march itself, state
handling (chunks, repeated read-outs, setting one beam of a batch) and the
refusal of the Lie-only entry points.
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import march as M
from oracle import turbulence as T
from paper_2306_15678_amd._lib import EUNSUPPORTED, SsfmError
from paper_2306_15678_amd.march import Propagator, desc_of

pytestmark = pytest.mark.gpu


def _strang(insts, precision, **kw):
    p = Propagator([desc_of(i) for i in insts], precision=precision, **kw)
    p.set_splitting(True)
    return p


def test_strang_matches_oracle_kerr():
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    ref = M.march(u0, inst, n_steps=100, strang=True)
    p = _strang([inst], 64)
    p.set_field(0, u0)
    p.propagate(100)
    err = M.rel_l2(p.field(0), ref.field)
    pw, pk = p.diag(0, 100)
    perr = float(np.max(np.abs(pw / ref.power - 1)))
    k0 = 2 * math.pi / inst.medium.wavelength
    half = M.propagator(inst.n, inst.length, inst.dz / 2, k0)
    want_peak = float(np.max(np.abs(M.diffract(ref.field, half)) ** 2))
    print(f"strang fp64 c1 field={err:.2e} power={perr:.2e} peak={abs(pk[-1] / want_peak - 1):.2e}",
          flush=True)
    # the Lie march of this beam meets the oracle to 2e-13 at step 100 (floors
    # of tests/golden/floor_c1.json); the Strang map has the same sensitivity
    assert err < 2e-13 and perr < 1e-12
    assert abs(pk[-1] / want_peak - 1) < 1e-12
    p.close()


def test_strang_matches_oracle_all_terms_with_screens():
    base = [b for b in W.config3() if b.n == 256][0]
    inst = dataclasses.replace(base, n_steps=60,
                               medium=dataclasses.replace(base.medium,
                                                          terms=base.medium.terms | W.TERM_ANSATZ),
                               theta=tuple(0.05 * np.abs(W.random_theta(4, 1.0))))
    u0 = W.initial_field(inst)
    ref = M.march(u0, inst, strang=True, screens=T.instance_screens(inst)).field
    p = _strang([inst], 64)
    p.gen_screens()
    p.set_field(0, u0)
    p.set_theta(0, np.array(inst.theta))
    p.propagate(inst.n_steps)
    err = M.rel_l2(p.field(0), ref)
    print(f"strang fp64 all terms + screen field={err:.2e}", flush=True)
    # the Lie march of this beam over 60 steps meets the oracle to 2.3e-14
    # (its per-step FP64 floor is 2.4e-14); 1e-12 is FP64 rounding here
    assert err < 1e-12
    p.close()


def test_strang_gpu_march_is_second_order():
    base = W.config1()[0]
    inst = dataclasses.replace(base, n=128, sigma=0.0)
    u0 = W.initial_field(inst)
    lz = 100 * base.dz

    def run(steps):
        i = dataclasses.replace(inst, dz=lz / steps)
        p = _strang([i], 64)
        p.set_field(0, u0)
        p.propagate(steps)
        f = p.field(0)
        p.close()
        return f

    ref = run(3200)
    # 50 steps is still pre-asymptotic here (ratio 3.66 against 3.95 next)
    errs = [np.linalg.norm(run(s) - ref) for s in (100, 200, 400)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    print(f"strang gpu order ratios {r1:.3f} {r2:.3f}", flush=True)
    assert 3.7 < r1 < 4.3 and 3.7 < r2 < 4.3


def test_strang_state_handling():
    insts = [W.config1()[0], W.config1()[0]]
    u0 = W.initial_field(insts[0])
    p = _strang(insts, 32)
    for b in range(2):
        p.set_field(b, u0)
    p.propagate(40)
    one = p.field(0)
    assert np.array_equal(p.field(0), one)          # a read-out leaves the state alone
    p.set_field(0, u0)
    p.set_field(1, u0)
    for _ in range(4):
        p.propagate(10)
    assert np.array_equal(p.field(0), one)          # chunks equal one march
    before = p.field(0)
    p.set_field(1, W.initial_field(insts[1]) * 0.5)  # the other beam is untouched
    assert np.array_equal(p.field(0), before)
    p.close()


def test_strang_mismatch_and_lens():
    """The fluence mismatch evaluates U = L(-dz/2) V: it equals the oracle's
    loss of its Strang march (and leaves the state alone); the effective
    lens, which would change U, is refused."""
    from paper_2306_15678_amd.march import make_lens
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 2)
    ref = M.march(u0, inst, n_steps=30, strang=True)
    p = _strang([inst], 64, max_steps=10, ckpt_every=5)
    p.set_field(0, u0)
    p.propagate(30)
    before = p.field(0)
    got = p.fluence_mismatch(0, target)
    want = M.fluence_loss(ref.field, target)[0]
    assert abs(got / want - 1) < 1e-11, (got, want)
    assert np.array_equal(p.field(0), before)
    with pytest.raises(SsfmError) as e:
        p.apply_lens(0, make_lens(0.0, 1.0, -1.0, 1e-12))
    assert e.value.status == EUNSUPPORTED
    p.close()


def test_strang_mixed_size_batch_equals_each_beam_alone():
    small = W.config1()[0]
    big = [b for b in W.config3() if b.n == 256][0]
    insts = [big, small]
    u = [W.initial_field(i) for i in insts]
    p = _strang(insts, 32)
    p.gen_screens()
    for k, x in enumerate(u):
        p.set_field(k, x)
    p.propagate(30)
    got = [p.field(k) for k in range(2)]
    p.close()
    for k, inst in enumerate(insts):
        q = _strang([inst], 32)
        q.gen_screens()
        q.set_field(0, u[k])
        q.propagate(30)
        assert np.array_equal(q.field(0), got[k])
        q.close()


def _grad_case(turb):
    """256^2, Kerr + MPA + plasma + ansatz, 200 P_cr, 8 steps; with
    turbulence, screens after steps 1, 4 and 7 (the last)."""
    terms = W.KPM | W.TERM_ANSATZ
    kw = {}
    if turb:
        terms |= W.TERM_TURB
        kw = dict(cn2=3e-13, screen_dz=0.03, n_screens=3)
    theta = tuple(np.array(W.THETA0) + W.random_theta(7, 0.1))
    return W.Instance(n=256, length=4e-3, dz=0.01, n_steps=8, medium=W.Medium(terms=terms),
                      w0=0.5e-3, power=200 * W.P_CR, sigma=0.2, seed=356, theta=theta, **kw)


def _strang_grads(inst, precision, ckpt, target):
    p = _strang([inst], precision, max_steps=inst.n_steps, ckpt_every=ckpt)
    if inst.medium.terms & W.TERM_TURB:
        p.gen_screens()
    p.set_field(0, W.initial_field(inst))
    p.set_theta(0, inst.theta)
    p.forward_record(inst.n_steps)
    loss = p.fluence_loss(0, target)
    p.backward()
    out = (loss, p.grad_field(0), p.grad_theta(0))
    p.close()
    return out


@pytest.mark.parametrize("turb", [False, True])
@pytest.mark.parametrize("precision,ckpt", [(64, 3), (64, 100), (32, 3)])
def test_strang_gradient_matches_oracle(precision, ckpt, turb):
    """The recorded Strang march and its adjoint against the oracle's Strang
    adjoint (checkpointed with recompute, M = 3, or all steps stored)."""
    inst = _grad_case(turb)
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    screens = T.instance_screens(inst) if turb else None
    loss, g_u0, g_th = M.gradient(u0, inst, screens=screens, strang=True,
                                  cotangent=lambda u: M.fluence_loss(u, target))
    gl, gg, gt = _strang_grads(inst, precision, ckpt, target)
    lerr = abs(gl / loss - 1)
    ferr = M.rel_l2(gg, g_u0)
    terr = float(np.max(np.abs(gt - g_th)) / np.max(np.abs(g_th)))
    print(f"strang grad fp{precision} M={ckpt} turb={turb}: loss {lerr:.2e} dL/dU0 {ferr:.2e} "
          f"dL/dtheta {terr:.2e}", flush=True)
    tol = 1e-10 if precision == 64 else 1e-4
    assert lerr < tol and ferr < tol and terr < tol


def test_strang_checkpointed_and_stored_adjoints_are_bitwise_equal():
    inst = _grad_case(True)
    target = W.synthetic_target(inst, 5)
    a = _strang_grads(inst, 32, 3, target)
    b = _strang_grads(inst, 32, 100, target)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_torch_autograd_through_a_strang_context():
    """autograd.march on a Strang context: a fluence loss written in torch,
    gradients in U0 and theta against the oracle's Strang adjoint."""
    import torch

    from paper_2306_15678_amd import autograd as AG

    inst = _grad_case(False)
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    _, g_u0, g_th = M.gradient(u0, inst, strang=True,
                               cotangent=lambda u: M.fluence_loss(u, target))
    dev = torch.device("cuda", 0)
    p = _strang([inst], 64, max_steps=inst.n_steps, ckpt_every=3)
    u = torch.from_numpy(u0).to(dev).requires_grad_(True)
    th = torch.tensor(inst.theta, dtype=torch.float64, requires_grad=True)
    t = torch.from_numpy(target).to(dev)
    out = AG.march(u, th, p, inst.n_steps)
    loss = torch.sum((out.abs() ** 2 - t) ** 2) / torch.sum(t ** 2)
    loss.backward()
    ferr = M.rel_l2(u.grad.cpu().numpy(), g_u0)
    terr = float(np.max(np.abs(th.grad.numpy() - g_th)) / np.max(np.abs(g_th)))
    print(f"strang autograd fp64: dL/dU0 {ferr:.2e} dL/dtheta {terr:.2e}", flush=True)
    assert ferr < 1e-10 and terr < 1e-10
    p.close()


def test_strang_full_size_matches_oracle():
    """The 1024^2 multifilamentation beam (Kerr, MPA, plasma), FP64, 20 Strang
    steps against the oracle's Strang march; FP32 against the same oracle at
    the FP32 rounding level of this short horizon."""
    inst = W.config2()[0]
    u0 = W.initial_field(inst)
    ref = M.march(u0, inst, n_steps=20, strang=True)
    for precision, tol in ((64, 1e-12), (32, 2e-5)):
        p = _strang([inst], precision)
        p.set_field(0, u0)
        p.propagate(20)
        err = M.rel_l2(p.field(0), ref.field)
        pw, _ = p.diag(0, 20)
        perr = float(np.max(np.abs(pw / ref.power - 1)))
        print(f"strang 1024^2 fp{precision} 20 steps: field={err:.2e} power={perr:.2e}", flush=True)
        assert err < tol and perr < tol
        p.close()
