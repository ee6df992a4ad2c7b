"""Pins of the oracle's effective-lens screen (Eq. (4)-(6))."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as D
from oracle import lens as LN


def test_filter_of_a_gaussian_is_the_wider_gaussian():
    """F^-1[exp(-l k^2) F exp(-2 r^2/w0^2)] = (w0^2/w1^2) exp(-2 r^2/w1^2),
    w1^2 = w0^2 + 8 l (the filter's k^2 and its normalisation)."""
    n, length, w0 = 256, 8e-3, 0.4e-3
    r2 = D.grid_r2(n, length)
    w = np.exp(-2 * r2 / w0 ** 2)
    for l_dif in (1e-9, 5e-9, 2e-8):
        w1sq = w0 ** 2 + 8 * l_dif
        want = (w0 ** 2 / w1sq) * np.exp(-2 * r2 / w1sq)
        got = LN.filtered_intensity(w, length, l_dif)
        assert np.max(np.abs(got - want)) < 1e-13


def test_zero_filter_is_the_identity():
    rng = np.random.default_rng(1)
    w = rng.random((64, 64))
    assert np.max(np.abs(LN.filtered_intensity(w, 1e-3, 0.0) - w)) < 1e-14


def test_profile_values():
    seg = [(1.0, 2.0, 3.0, 0.5), (2.5, -1.0, 0.0, 0.0)]
    r = np.array([0.0, 0.5, 0.999, 1.0, 2.0, 2.5, 3.0])
    want = [2 * math.cos(0.5), 2 * math.cos(2.0), 2 * math.cos(3.497), -1.0, -1.0, 0.0, 0.0]
    assert np.allclose(LN.profile(r, seg), want, rtol=0, atol=1e-15)


def test_radius_inverts_the_cubic():
    c1, c2 = -3e21, 2.7e-10          # w = c1 (r^3 - c2) falls from 8.1e11 to 0 at r = 0.646 mm
    r0 = np.linspace(0, 6e-4, 101)
    w = c1 * (r0 ** 3 - c2)
    assert np.max(np.abs(LN.radius(w, c1, c2) - r0)) < 1e-15
    assert np.all(LN.radius(np.array([c1 * (-c2) * 2]), c1, c2) == 0.0)  # above the centre value


def _field():
    inst = W.config1()[0]
    return inst, W.initial_field(inst)


def _lens(inst, u, absorb):
    w = np.abs(u) ** 2
    peak = float(w.max())
    return LN.Lens(l_dif=(inst.length / inst.n) ** 2 * 4, w_l=0.3 * peak, c1=-peak / (4e-4) ** 3,
                   c2=(4e-4) ** 3,
                   re=[(2e-4, 0.8, 5e3, 0.0), (4e-4, 0.4, 1e4, 0.3)],
                   im=[(3e-4, 0.05 if absorb else 0.0, 2e3, 0.0)])


def test_phase_only_lens_keeps_the_intensity_and_untouched_points():
    inst, u = _field()
    lens = _lens(inst, u, absorb=False)
    v = LN.apply_lens(u, inst.length, lens)
    assert np.allclose(np.abs(v), np.abs(u), rtol=1e-15, atol=0)
    _, _, active = LN.lens_exponent(u, inst.length, lens)
    assert 0 < active.sum() < active.size
    assert np.array_equal(v[~active], u[~active])
    assert not np.allclose(v[active], u[active])


def test_absorbing_lens_lowers_the_power():
    inst, u = _field()
    v = LN.apply_lens(u, inst.length, _lens(inst, u, absorb=True))
    assert np.sum(np.abs(v) ** 2) < np.sum(np.abs(u) ** 2)


def _smooth_lens(inst, u):
    """A lens whose f is continuous: one segment per part ending at r_end with
    cos(...) = 0 there, trimming beyond r_end (r in [0.238, 0.29] mm on the
    active points), so finite differences see no jump."""
    peak = float(LN.filtered_intensity(np.abs(u) ** 2, inst.length,
                                       4 * (inst.length / inst.n) ** 2).max())
    c2 = (0.3e-3) ** 3
    r_end, om, nu = 0.28e-3, 2.0e4, 1.0e4
    return LN.Lens(4 * (inst.length / inst.n) ** 2, 0.2 * peak, -2.0 * peak / c2, c2,
                   [(r_end, 0.7, om, math.pi / 2 - om * r_end)],
                   [(r_end, 0.05, nu, math.pi / 2 - nu * r_end)])


def _functional(u, g, length, lens):
    return float(np.real(np.sum(np.conj(g) * LN.apply_lens(u, length, lens))))


def test_lens_vjp_field_cotangent_matches_finite_differences():
    inst, u = _field()
    lens = _smooth_lens(inst, u)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    d = (rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)) * np.abs(u).max()
    g_in, _ = LN.lens_vjp(u, g, inst.length, lens)
    want = float(np.real(np.sum(np.conj(g_in) * d)))
    for h in (1e-5, 5e-6):
        fd = (_functional(u + h * d, g, inst.length, lens)
              - _functional(u - h * d, g, inst.length, lens)) / (2 * h)
        assert abs(fd / want - 1) < 1e-6, (h, fd, want)
    # the nonlocal part (through the filtered intensity) carries a share of
    # the derivative far above the tolerance, so an error in it shows
    f_re, f_im, act = LN.lens_exponent(u, inst.length, lens)
    local = np.where(act, np.exp(-f_im) * np.exp(-1j * f_re), 1.0) * g
    share = float(np.real(np.sum(np.conj(g_in - local) * d))) / want
    assert abs(share) > 1e-3, share


def test_lens_vjp_parameter_gradients_match_finite_differences():
    inst, u = _field()
    lens = _smooth_lens(inst, u)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    _, grad = LN.lens_vjp(u, g, inst.length, lens)
    names = ["c1", "c2", "re.a", "re.omega", "re.psi", "im.b", "im.nu", "im.eta"]

    def with_param(k, v):
        c1, c2 = lens.c1, lens.c2
        re, im = [list(s) for s in lens.re], [list(s) for s in lens.im]
        if k == 0:
            c1 = v
        elif k == 1:
            c2 = v
        elif k < 5:
            re[0][k - 1] = v
        else:
            im[0][k - 4] = v
        return LN.Lens(lens.l_dif, lens.w_l, c1, c2, [tuple(s) for s in re], [tuple(s) for s in im])

    base = [lens.c1, lens.c2, *lens.re[0][1:], *lens.im[0][1:]]
    for k, name in enumerate(names):
        h = 1e-6 * abs(base[k])
        fd = (_functional(u, g, inst.length, with_param(k, base[k] + h))
              - _functional(u, g, inst.length, with_param(k, base[k] - h))) / (2 * h)
        assert abs(fd - grad[k]) < 1e-5 * abs(grad[k]) + 1e-12, (name, fd, grad[k])
        assert abs(grad[k]) > 0, name
