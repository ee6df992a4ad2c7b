"""GPU effective-lens screen against the oracle (Eq. (4)-(6)).

The GPU filters |U|^2 with its separable row/column pass kernels, the
oracle with a 2-D FFT; both then trim, invert the cubic and apply the
piecewise-cosine profile.  FP64: the same field to rounding.  FP32: a
profile that vanishes smoothly where it ends (as the paper's smoothness
requirement asks), so rounding near the trim level or a segment end moves
f by rounding only.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lens as LN
from paper_2306_15678_amd._lib import EINVAL, ESTATE, SsfmError
from paper_2306_15678_amd.march import Propagator, desc_of, make_lens, march_with_lens

pytestmark = pytest.mark.gpu


def _prop(insts, precision, **kw):
    return Propagator([desc_of(i) for i in insts], precision=precision, **kw)


def _lens_params(inst, u, smooth):
    """A lens scaled to the filtered intensity w_dif of u: the cubic lens
    field reaches 2 x max(w_dif) at its centre and 0 at r = 0.3 mm, the
    trimming level is 0.2 x max(w_dif), so every active point has r in
    [0.238, 0.290] mm, away from the cube root's singular point r = 0."""
    l_dif = 4 * (inst.length / inst.n) ** 2
    peak = float(LN.filtered_intensity(np.abs(u) ** 2, inst.length, l_dif).max())
    c2 = (0.3e-3) ** 3
    c1 = -2.0 * peak / c2
    w_l = 0.2 * peak
    if smooth:
        # one segment per part ending at r_end with cos(...) = 0 there
        r_end = 0.28e-3
        om, nu = 2.0e4, 1.0e4
        re = [(r_end, 0.7, om, math.pi / 2 - om * r_end)]
        im = [(r_end, 0.05, nu, math.pi / 2 - nu * r_end)]
    else:
        re = [(0.25e-3, 0.8, 1.5e4, 0.2), (0.275e-3, -0.3, 4e3, 0.0)]
        im = [(0.26e-3, 0.1, 5e3, 0.0)]
    return LN.Lens(l_dif, w_l, c1, c2, re, im)


def _to_gpu(lens):
    return make_lens(lens.l_dif, lens.w_l, lens.c1, lens.c2, lens.re, lens.im)


@pytest.mark.parametrize("precision,smooth,tol", [(64, False, 1e-12), (64, True, 1e-12),
                                                  (32, True, 2e-5)])
def test_lens_matches_oracle(precision, smooth, tol):
    inst = W.config1()[0]
    p = _prop([inst], precision)
    p.set_field(0, W.initial_field(inst))
    p.propagate(100)
    u = p.field(0)
    lens = _lens_params(inst, u, smooth)
    p.apply_lens(0, _to_gpu(lens))
    got = p.field(0)
    want = LN.apply_lens(u, inst.length, lens)
    _, _, active = LN.lens_exponent(u, inst.length, lens)
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    moved = float(np.linalg.norm(want - u) / np.linalg.norm(u))
    print(f"lens fp{precision} smooth={smooth} err={err:.2e} lens moved the field by {moved:.2e} "
          f"on {int(active.sum())} points", flush=True)
    assert 0 < active.sum() < active.size and moved > 1e-3
    assert err < tol
    p.close()


def test_lens_touches_only_its_instance():
    insts = [W.config1()[0], W.config1()[0]]
    p = _prop(insts, 32)
    for b in range(2):
        p.set_field(b, W.initial_field(insts[b]))
    p.propagate(80)
    before = [p.field(b) for b in range(2)]
    p.apply_lens(1, _to_gpu(_lens_params(insts[1], before[1], True)))
    assert np.array_equal(p.field(0), before[0])
    assert not np.array_equal(p.field(1), before[1])
    p.close()


def test_march_with_lens_triggers_at_the_pre_filamentation_level():
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    p = _prop([inst], 32)
    p.set_field(0, u0)
    p.propagate(60)
    peak0 = float(p.diag(0, 60)[1].max())
    w_pf = 2.0 * peak0
    lens = _to_gpu(_lens_params(inst, p.field(0), True))
    p.set_field(0, u0)
    at = march_with_lens(p, 0, 200, w_pf, lens, chunk=20)
    got = p.field(0)
    # the same by hand
    p.set_field(0, u0)
    manual = None
    for k in range(10):
        p.propagate(20)
        if manual is None and float(p.diag(0, 20)[1].max()) >= w_pf:
            p.apply_lens(0, lens)
            manual = 20 * (k + 1)
    assert at == manual and at is not None
    assert np.array_equal(got, p.field(0))
    p.close()


def test_lens_ends_the_recorded_march_and_rejects_bad_parameters():
    inst = W.config1()[0]
    p = _prop([inst], 32, max_steps=20, ckpt_every=10)
    p.set_field(0, W.initial_field(inst))
    p.forward_record(20)
    lens = _lens_params(inst, p.field(0), True)
    p.apply_lens(0, _to_gpu(lens))
    with pytest.raises(SsfmError) as e:
        p.set_cotangent(0, np.zeros((inst.n, inst.n), complex))
        p.backward()
    assert e.value.status == ESTATE
    bad = _to_gpu(LN.Lens(lens.l_dif, lens.w_l, lens.c1, lens.c2,
                          [(2e-4, 1, 1, 0), (1e-4, 1, 1, 0)], []))
    with pytest.raises(SsfmError) as e:
        p.apply_lens(0, bad)
    assert e.value.status == EINVAL
    with pytest.raises(SsfmError) as e:
        p.apply_lens(0, _to_gpu(LN.Lens(-1.0, 0, -1, 0, [], [])))
    assert e.value.status == EINVAL
    p.close()


def _vjp_setup(precision):
    inst = W.config1()[0]
    p = _prop([inst], precision, max_steps=40, ckpt_every=10)
    p.set_field(0, W.initial_field(inst))
    p.propagate(100)
    u = p.field(0)
    return inst, p, u, _lens_params(inst, u, True)


@pytest.mark.parametrize("precision,tol_g,tol_p", [(64, 1e-12, 1e-11), (32, 2e-5, 1e-4)])
def test_lens_vjp_matches_oracle(precision, tol_g, tol_p):
    inst, p, u, lens = _vjp_setup(precision)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    g_in, grad = p.lens_vjp(0, _to_gpu(lens), u, g)
    want_g, want_p = LN.lens_vjp(u, g, inst.length, lens)
    err_g = float(np.linalg.norm(g_in.cpu().numpy() - want_g) / np.linalg.norm(want_g))
    err_p = np.abs(grad - want_p) / np.abs(want_p)
    print(f"lens vjp fp{precision}: g_in {err_g:.2e}, parameter gradients max rel "
          f"{err_p.max():.2e} ({len(grad)} values)", flush=True)
    assert err_g < tol_g and err_p.max() < tol_p
    # the context's own field is untouched
    assert np.array_equal(p.field(0), u)
    p.close()


def test_lens_vjp_composes_with_the_recorded_march():
    """FP64: march 60 steps -> lens -> recorded march 20 steps -> fluence
    loss.  backward gives the cotangent at the lens output, lens_vjp the
    lens-parameter gradients and the cotangent at its input, a re-recorded
    first march with that cotangent the gradient in the initial field; all
    against central finite differences of the whole pipeline."""
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 3)
    p = _prop([inst], 64, max_steps=60, ckpt_every=20)
    p.set_field(0, u0)
    p.propagate(60)
    u1 = p.field(0)
    base = _lens_params(inst, u1, True)

    def loss(lens, start=u0):
        p.set_field(0, start)
        p.propagate(60)
        p.apply_lens(0, _to_gpu(lens))
        p.forward_record(20)
        return p.fluence_loss(0, target)

    loss(base)
    p.backward()
    g_out = p.grad_field(0)
    g_in, grad = p.lens_vjp(0, _to_gpu(base), u1, g_out)
    # parameters: c2, the real amplitude and the imaginary frequency
    for k, name in ((1, "c2"), (2, "re.a"), (6, "im.nu")):
        vals = [base.c1, base.c2, *base.re[0][1:], *base.im[0][1:]]
        h = 1e-6 * abs(vals[k])

        def shifted(dv):
            v = list(vals)
            v[k] += dv
            return LN.Lens(base.l_dif, base.w_l, v[0], v[1], [(base.re[0][0], v[2], v[3], v[4])],
                           [(base.im[0][0], v[5], v[6], v[7])])

        fd = (loss(shifted(h)) - loss(shifted(-h))) / (2 * h)
        print(f"lens gradient {name}: adjoint {grad[k]:.6e} finite difference {fd:.6e}", flush=True)
        assert abs(fd / grad[k] - 1) < 1e-5
    # the initial field, through the lens input cotangent
    p.set_field(0, u0)
    p.forward_record(60)
    p.set_cotangent(0, g_in)
    p.backward()
    g0 = p.grad_field(0)
    d = np.random.default_rng(5).standard_normal(u0.shape) * np.abs(u0)
    h = 1e-6
    fd = (loss(base, u0 + h * d) - loss(base, u0 - h * d)) / (2 * h)
    adj = float(np.real(np.sum(np.conj(g0) * d)))
    print(f"dL/dU0 along a direction: adjoint {adj:.6e} finite difference {fd:.6e}", flush=True)
    assert abs(fd / adj - 1) < 1e-5
    p.close()


def test_lens_without_segments_has_an_identity_vjp():
    """No profile segments: f = 0 everywhere, so E = 1, the input cotangent
    is the output cotangent and the two gradients (c1, c2) vanish."""
    inst, p, u, lens = _vjp_setup(64)
    empty = LN.Lens(lens.l_dif, lens.w_l, lens.c1, lens.c2, [], [])
    g = np.random.default_rng(8).standard_normal(u.shape) + 0j
    g_in, grad = p.lens_vjp(0, _to_gpu(empty), u, g)
    assert np.array_equal(g_in.cpu().numpy(), g) and len(grad) == 2 and not grad.any()
    p.close()


def test_torch_autograd_through_march_lens_march():
    """march 60 -> lens -> march 20 -> a fluence loss written in torch, all
    through torch autograd (two contexts, FP64): gradients of two lens
    parameters and of U0 along a direction against central differences."""
    import torch

    from paper_2306_15678_amd import autograd as AG

    inst = W.config1()[0]
    dev = torch.device("cuda", 0)
    u0 = torch.from_numpy(W.initial_field(inst)).to(dev)
    target = torch.from_numpy(W.synthetic_target(inst, 3)).to(dev)
    theta = torch.zeros(8, dtype=torch.float64)
    p1 = _prop([inst], 64, max_steps=60, ckpt_every=20)
    p2 = _prop([inst], 64, max_steps=20, ckpt_every=20)
    p1.set_field(0, u0)
    p1.propagate(60)
    template = _to_gpu(_lens_params(inst, p1.field(0), True))
    base = AG.lens_params_vector(template)

    def pipeline(u, params):
        u1 = AG.march(u, theta, p1, 60)
        u2 = AG.lens(u1, params, p2, 0, template)
        u3 = AG.march(u2, theta, p2, 20)
        return torch.sum((u3.abs() ** 2 - target) ** 2) / torch.sum(target ** 2)

    u = u0.clone().requires_grad_(True)
    params = torch.tensor(base, dtype=torch.float64, requires_grad=True)
    pipeline(u, params).backward()
    with torch.no_grad():
        for k, name in ((1, "c2"), (2, "re.a")):
            h = 1e-6 * abs(base[k])
            up, dn = list(base), list(base)
            up[k] += h
            dn[k] -= h
            fd = (pipeline(u0, torch.tensor(up, dtype=torch.float64))
                  - pipeline(u0, torch.tensor(dn, dtype=torch.float64))).item() / (2 * h)
            got = params.grad[k].item()
            print(f"torch lens gradient {name}: autograd {got:.6e} finite difference {fd:.6e}",
                  flush=True)
            assert abs(fd / got - 1) < 1e-5
        d = torch.from_numpy(np.random.default_rng(6).standard_normal(u0.shape)).to(dev) * u0.abs()
        h = 1e-6
        p_base = torch.tensor(base, dtype=torch.float64)
        fd = (pipeline(u0 + h * d, p_base) - pipeline(u0 - h * d, p_base)).item() / (2 * h)
        adj = torch.sum(torch.real(torch.conj(u.grad) * d)).item()
        print(f"torch dL/dU0 along a direction: autograd {adj:.6e} finite difference {fd:.6e}",
              flush=True)
        assert abs(fd / adj - 1) < 1e-5
    p1.close()
    p2.close()


def test_lens_vjp_at_1024():
    """The lens and its VJP on the 1024^2 multifilamentation field after 200
    steps (FP64), lens scaled to its filtered intensity: against the oracle."""
    inst = W.config2()[0]
    p = _prop([inst], 64)
    p.set_field(0, W.initial_field(inst))
    p.propagate(200)
    u = p.field(0)
    lens = _lens_params(inst, u, True)
    g = np.random.default_rng(9).standard_normal(u.shape) + 0.5j
    g_in, grad = p.lens_vjp(0, _to_gpu(lens), u, g)
    want_g, want_p = LN.lens_vjp(u, g, inst.length, lens)
    err_g = float(np.linalg.norm(g_in.cpu().numpy() - want_g) / np.linalg.norm(want_g))
    err_p = float(np.max(np.abs(grad - want_p) / np.abs(want_p)))
    _, _, active = LN.lens_exponent(u, inst.length, lens)
    print(f"lens vjp 1024^2 fp64: g_in {err_g:.2e}, gradients {err_p:.2e}, "
          f"{int(active.sum())} active points", flush=True)
    assert active.sum() > 0 and err_g < 1e-12 and err_p < 1e-10
    p.close()
