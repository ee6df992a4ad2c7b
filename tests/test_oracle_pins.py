"""Pins of the FP64 oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: a brute-force
DFT, the Gaussian-beam closed form, plane-wave closed forms, invariants,
symmetry, the convergence order of Lie splitting, and (for the adjoint)
finite differences and an independent autodiff of the same map.
"""
import dataclasses
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import march as M

HERE = os.path.dirname(os.path.abspath(__file__))


def _inst(n=32, length=4e-3, dz=2e-3, terms=W.TERM_KERR, theta=None, **kw):
    base = dict(n=n, length=length, dz=dz, n_steps=10,
                medium=W.Medium(terms=terms), w0=0.6e-3, power=5 * W.P_CR,
                sigma=0.05, seed=7, theta=theta)
    base.update(kw)
    return W.Instance(**base)


# --------------------------------------------------------------- P1: DFT
@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_diffraction_matches_brute_force_dft(n):
    """V = F^-1 P F U against explicit O(N^4) DFT sums with the paraxial
    propagator exp(-i k^2 dz / 2k0) built from signed integer frequencies."""
    rng = np.random.default_rng(n)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    length, dz, k0 = 1e-3, 0.37, W.K0
    prop = M.propagator(n, length, dz, k0)
    got = M.diffract(u, prop)
    idx = np.arange(n)
    signed = np.where(idx <= n // 2, idx, idx - n)
    kvec = 2 * math.pi * signed / length
    want = np.zeros((n, n), complex)
    for ky in range(n):
        for kx in range(n):
            fk = 0j
            for y in range(n):
                for x in range(n):
                    fk += u[y, x] * np.exp(-2j * math.pi * (kx * x + ky * y) / n)
            fk *= np.exp(-1j * (kvec[kx] ** 2 + kvec[ky] ** 2) * dz / (2 * k0))
            for y in range(n):
                for x in range(n):
                    want[y, x] += fk * np.exp(2j * math.pi * (kx * x + ky * y) / n)
    want /= n * n
    assert M.rel_l2(got, want) < 1e-13


# ------------------------------------------------------ P2: Gaussian beam
def _gauss_exact(n, length, w0, z, k0, images=2):
    x = W.grid_axis(n, length)
    zr = k0 * w0 ** 2 / 2
    q = 1 + 1j * z / zr
    out = np.zeros((n, n), complex)
    for iy in range(-images, images + 1):
        for ix in range(-images, images + 1):
            xx = x[None, :] - ix * length
            yy = x[:, None] - iy * length
            out += np.exp(-(xx ** 2 + yy ** 2) / (w0 ** 2 * q)) / q
    return out


def test_linear_step_matches_gaussian_closed_form():
    """n2 = 0: the periodic sum of exp(-r^2/(w0^2 q))/q, q = 1 + i z/z_R,
    z_R = k0 w0^2/2, solves dU/dz = (i/2k0) Lap U exactly."""
    n, length, w0 = 64, 8e-3, 1e-3
    inst = _inst(n=n, length=length, dz=0.05, terms=0, w0=w0)
    u0 = _gauss_exact(n, length, w0, 0.0, W.K0)
    res = M.march(u0, inst, n_steps=40)
    want = _gauss_exact(n, length, w0, 40 * 0.05, W.K0)
    assert M.rel_l2(res.field, want) < 1e-13


def test_second_moment_width_follows_rayleigh_law():
    """w(z) = sqrt(2 <r^2>) = w0 sqrt(1 + (z/z_R)^2) (linear diffraction)."""
    n, length, w0 = 128, 16e-3, 1e-3
    zr = W.K0 * w0 ** 2 / 2
    inst = _inst(n=n, length=length, dz=zr / 20, terms=0, w0=w0)
    u0 = W.gaussian_beam(n, length, w0, 1.0, 0.0, 0)
    x = W.grid_axis(n, length)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    res = M.march(u0, inst, n_steps=30)
    inten = np.abs(res.field) ** 2
    w_num = math.sqrt(2 * np.sum(r2 * inten) / np.sum(inten))
    w_th = w0 * math.sqrt(1 + (30 * inst.dz / zr) ** 2)
    assert abs(w_num / w_th - 1) < 1e-10


# ---------------------------------------------------- P3: plane-wave modes
def test_plane_wave_mode_is_eigenvector():
    n, length, dz = 16, 2e-3, 0.3
    x = np.arange(n) * (length / n)
    m = 3
    k = 2 * math.pi * m / length
    u = np.exp(1j * k * x)[None, :] * np.ones((n, 1))
    v = M.diffract(u, M.propagator(n, length, dz, W.K0))
    assert np.max(np.abs(v - u * np.exp(-1j * k * k * dz / (2 * W.K0)))) < 1e-13


# ------------------------------------- P4/P5: uniform plane-wave screens
def test_uniform_wave_phase_closed_form():
    """A uniform wave only picks up its own nonlinear phase per step."""
    theta = W.random_theta(3)
    terms = W.TERM_KERR | W.TERM_PLASMA | W.TERM_ANSATZ
    inst = _inst(n=8, terms=terms, theta=tuple(theta))
    # ansatz imaginary part makes an amplitude change; drop it for this pin
    th = np.array(theta)
    th[4:] = 0.0
    i0 = 0.8 * W.I_A
    u0 = np.full((8, 8), math.sqrt(i0), complex)
    res = M.march(u0, inst, n_steps=7, theta=th)
    x = i0 / W.I_A
    kn = W.K0 * W.N2 * inst.dz
    re = sum(th[p - 1] * x ** p for p in range(1, 5)) / (1 + x ** 4)
    phi = kn * i0 - kn * W.I_A * x ** 8 / (1 + x ** 7) + kn * W.I_A * re
    want = math.sqrt(i0) * np.exp(1j * 7 * phi)
    assert np.max(np.abs(res.field - want)) / math.sqrt(i0) < 1e-13


def test_uniform_wave_mpa_exact_solution():
    """I(z) = I0 (1 + (K-1) beta I0^(K-1) z)^(-1/(K-1)) at any dz."""
    inst = _inst(n=8, dz=0.37, terms=W.TERM_MPA)
    i0 = 3.0 * W.I_A
    u0 = np.full((8, 8), math.sqrt(i0), complex)
    res = M.march(u0, inst, n_steps=9)
    K, b = W.K_MPA, W.BETA_K
    for n in range(9):
        z = (n + 1) * inst.dz
        want = i0 * (1 + (K - 1) * b * i0 ** (K - 1) * z) ** (-1 / (K - 1))
        assert abs(res.peak[n] / want - 1) < 1e-13


# --------------------------------------------------------- P6: invariants
def test_power_conserved_without_absorption():
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    res = M.march(u0, inst, n_steps=200)
    p0 = inst.power
    for n in range(200):
        assert abs(res.power[n] / p0 - 1) < 1e-13 * math.sqrt(n + 1) + 1e-15


def test_energy_balance_with_mpa():
    """P_{n+1} = sum |V|^2 A^2 dx^2 with A the exact MPA amplitude."""
    inst = _inst(n=32, terms=W.KPM, dz=0.05)
    u0 = W.gaussian_beam(32, inst.length, inst.w0, 200 * W.P_CR, 0.05, 1)
    res = M.march(u0, inst, n_steps=3, keep_pre_screen=True)
    K, b = W.K_MPA, W.BETA_K
    for n in range(3):
        i = np.abs(res.pre_screen[n]) ** 2
        a2 = (1 + (K - 1) * b * i ** (K - 1) * inst.dz) ** (-1 / (K - 1))
        want = np.sum(i * a2) * inst.dx ** 2
        assert abs(res.power[n] / want - 1) < 1e-13
    assert res.power[-1] < res.power[0] < 200 * W.P_CR


# ---------------------------------------------------------- P7: symmetry
def test_shift_and_transpose_commute_with_march():
    inst = _inst(n=32, terms=W.KPM, dz=0.05)
    u0 = W.gaussian_beam(32, inst.length, inst.w0, 150 * W.P_CR, 0.1, 2)
    base = M.march(u0, inst, n_steps=5).field
    shifted = M.march(np.roll(u0, (3, -5), axis=(0, 1)), inst, n_steps=5).field
    assert M.rel_l2(shifted, np.roll(base, (3, -5), axis=(0, 1))) < 1e-12
    tr = M.march(u0.T.copy(), inst, n_steps=5).field
    assert M.rel_l2(tr, base.T) < 1e-12


def test_mirror_even_input_stays_even():
    inst = _inst(n=32, terms=W.KPM, dz=0.05)
    u0 = W.gaussian_beam(32, inst.length, inst.w0, 150 * W.P_CR, 0.0, 0)
    # cell-centred grid: x -> -x maps index j to n-1-j
    res = M.march(u0, inst, n_steps=5).field
    assert M.rel_l2(res[:, ::-1], res) < 1e-12
    assert M.rel_l2(res[::-1, :], res) < 1e-12


# ------------------------------------------------- P8: splitting order
@pytest.mark.slow
def test_lie_splitting_is_first_order():
    base = W.config1()[0]
    inst = dataclasses.replace(base, n=64, sigma=0.0)
    u0 = W.initial_field(inst)
    lz = 200 * base.dz

    def run(steps):
        return M.march(u0, dataclasses.replace(inst, dz=lz / steps),
                       n_steps=steps).field

    ref = run(64 * 64)
    errs = [np.linalg.norm(run(s) - ref) for s in (32, 64, 128)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.9 < r1 < 2.1 and 1.9 < r2 < 2.1


def test_strang_splitting_is_second_order():
    base = W.config1()[0]
    inst = dataclasses.replace(base, n=64, sigma=0.0)
    u0 = W.initial_field(inst)
    lz = 200 * base.dz

    def run(steps):
        return M.march(u0, dataclasses.replace(inst, dz=lz / steps), n_steps=steps,
                       strang=True).field

    ref = run(64 * 64)
    errs = [np.linalg.norm(run(s) - ref) for s in (64, 128, 256)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, (r1, r2)


def test_strang_step_is_time_reversible():
    """With a phase-only screen the Strang step is symmetric: n steps of dz
    followed by n steps of -dz return U0 (the Lie step is not)."""
    inst = dataclasses.replace(W.config1()[0], n=64,
                               medium=W.Medium(terms=W.TERM_KERR | W.TERM_PLASMA))
    u0 = W.initial_field(inst)
    back = dataclasses.replace(inst, dz=-inst.dz)
    fwd = M.march(u0, inst, n_steps=40, strang=True).field
    ret = M.march(fwd, back, n_steps=40, strang=True).field
    assert M.rel_l2(ret, u0) < 1e-12
    lie = M.march(M.march(u0, inst, n_steps=40).field, back, n_steps=40).field
    assert M.rel_l2(lie, u0) > 1e-6


def test_strang_without_nonlinearity_is_the_linear_propagator():
    inst = dataclasses.replace(W.config1()[0], n=64, medium=W.Medium(terms=0))
    u0 = W.initial_field(inst)
    s = M.march(u0, inst, n_steps=7, strang=True).field
    lie = M.march(u0, inst, n_steps=7).field
    assert M.rel_l2(s, lie) < 1e-14


def test_virial_identity_fixes_kerr_strength():
    """Kerr-only NLS: V(z) = int r^2 |U|^2 is exactly quadratic in z,
    V(z) = (P w0^2/2) (1 + (z/z_R)^2 (1 - P/P_G)), P_G = lambda^2/(2 pi n2)
    (variance identity).  A wrong Kerr coefficient or diffraction constant
    changes the curvature; the split-step error is O(dz)."""
    inst = dataclasses.replace(W.config1()[0], n=128, sigma=0.0, dz=2e-3)
    u0 = W.initial_field(inst)
    x = W.grid_axis(inst.n, inst.length)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    zr = W.rayleigh_length(inst.w0)
    p_g = W.LAMBDA ** 2 / (2 * math.pi * W.N2)
    u = u0
    for k in range(1, 4):
        u = M.march(u, inst, n_steps=100).field
        z = 100 * k * inst.dz
        v = np.sum(r2 * np.abs(u) ** 2) * inst.dx ** 2
        want = inst.power * inst.w0 ** 2 / 2 * (
            1 + (z / zr) ** 2 * (1 - inst.power / p_g))
        assert abs(v / want - 1) < 5e-3


def test_kerr_collapse_precedes_virial_bound():
    """Loose physics sanity, not a parity pin: the collimated 5 P_cr beam
    collapses before z_R / sqrt(P/P_G - 1) ~ 2.05 m; Marburger's fit in the
    form 0.367 z_R / sqrt((sqrt(P/P_cr) - 0.852)^2 - 0.0219) gives 1.05 m."""
    inst = dataclasses.replace(W.config1()[0], n=128, sigma=0.0, dz=5e-3)
    u0 = W.initial_field(inst)
    res = M.march(u0, inst, n_steps=400)
    z30 = (int(np.argmax(res.peak > 30 * res.peak[0])) + 1) * inst.dz
    zr = W.rayleigh_length(inst.w0)
    p_g = W.LAMBDA ** 2 / (2 * math.pi * W.N2)
    z_var = zr / math.sqrt(inst.power / p_g - 1)
    z_m = 0.367 * zr / math.sqrt((math.sqrt(5) - 0.852) ** 2 - 0.0219)
    assert z30 < z_var
    assert abs(z30 / z_m - 1) < 0.1


# ------------------------------------------------------------ ansatz fit
def test_theta0_matches_fit_script():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_theta0", os.path.join(HERE, "golden", "make_theta0.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    fit = mod.fit_theta0()
    assert np.allclose(fit, np.array(W.THETA0), rtol=1e-7, atol=1e-7)


# --------------------------------------------- loss pieces on hand arrays
def test_block_mean_of_hand_built_array():
    """8 x 8 block means of the dense fluence onto the sparse grid (the
    discrepancy target): rows are y, columns x; a transposed or mis-strided
    reshape moves the values below."""
    w = np.arange(1.0, 17.0).reshape(4, 4)
    assert np.array_equal(M.block_mean(w, 2), np.array([[3.5, 5.5], [11.5, 13.5]]))
    w6 = np.zeros((6, 6))
    w6[0:3, 3:6] = 9.0          # top right block (y < 3, x >= 3)
    w6[4, 1] = 18.0             # one point in the bottom left block
    assert np.array_equal(M.block_mean(w6, 3), np.array([[0.0, 9.0], [2.0, 0.0]]))
    assert np.array_equal(M.block_mean(w6, 1), w6)
    assert M.block_mean(w6, 6)[0, 0] == pytest.approx(w6.mean(), rel=1e-15)


def test_fluence_loss_value_and_cotangent_on_a_2x2_case():
    """L = sum (|U|^2 - w)^2 / sum w^2 and G = 4 (|U|^2 - w) U / sum w^2 by
    hand: |U|^2 = [[1, 1], [4, 0]], w = [[2, 1], [1, 1]], so the mismatch
    is [[-1, 0], [3, -1]], L = 11/7 and G = [[-4/7, 0], [24/7, 0]]."""
    u = np.array([[1.0, 1j], [2.0, 0.0]])
    w = np.array([[2.0, 1.0], [1.0, 1.0]])
    loss, g = M.fluence_loss(u, w)
    assert loss == pytest.approx(11.0 / 7.0, rel=1e-15)
    assert np.allclose(g, np.array([[-4.0 / 7.0, 0.0], [24.0 / 7.0, 0.0]]), rtol=0, atol=1e-15)
    # the normalisation: scaling the target and |U|^2 together leaves L
    l2, _ = M.fluence_loss(3.0 * u, 9.0 * w)
    assert l2 == pytest.approx(loss, rel=1e-14)
    assert M.fluence_loss(u, np.abs(u) ** 2 + 0.0)[0] == 0.0


# ------------------------------ R9: saturating plasma, by its own properties
def _phase_per_unit(terms, x):
    """Phase of one step divided by k0 n2 I_a dz, at x = I / I_a."""
    inst = _inst(terms=terms)
    scr = M.Screen.of(inst)
    ph, dph = scr.phase(np.asarray(x, dtype=float) * W.I_A)
    kn = scr.k0 * scr.n2 * scr.dz
    return ph / (kn * W.I_A), dph / kn


def test_saturating_plasma_caps_the_total_index():
    """With the plasma term Kerr + plasma is n2 I / (1 + x^(K-1)) (K = 8):
    it peaks at x* = 6^(-1/7) with the value (6/7) 6^(-1/7) = 0.6636 n2 I_a,
    the reading's bounded per-step phase.  An exponent off by one, a dropped
    I_a or a sign flip moves the peak or removes it."""
    kp = W.TERM_KERR | W.TERM_PLASMA
    xs = 6.0 ** (-1.0 / 7.0)
    ph, dph = _phase_per_unit(kp, [xs])
    assert xs == pytest.approx(0.77417, abs=1e-5)
    assert ph[0] == pytest.approx(6.0 / 7.0 * xs, rel=1e-14)
    assert ph[0] == pytest.approx(0.6636, abs=1e-4)
    assert abs(dph[0]) < 1e-13              # stationary at x*
    grid = np.linspace(0.0, 5.0, 50001)
    g, _ = _phase_per_unit(kp, grid)
    assert g.max() <= ph[0] * (1 + 1e-15)
    assert grid[np.argmax(g)] == pytest.approx(xs, abs=1e-4)
    # above the peak the index falls like x^-(K-2): x/(1+x^7) at x = 4 over x = 2
    big, _ = _phase_per_unit(kp, [2.0, 4.0])
    assert big[1] / big[0] == pytest.approx(2.0 * 129.0 / 16385.0, rel=1e-12)


def test_plasma_term_scales_as_i_to_the_k_at_low_intensity():
    """The plasma phase alone is -x^K/(1 + x^(K-1)) per unit: at low
    intensity the power law of Eq. (3) with K = 8 and a negative sign."""
    ph, _ = _phase_per_unit(W.TERM_PLASMA, [1e-3, 2e-3])
    assert ph[0] < 0 and ph[1] < 0
    slope = math.log(ph[1] / ph[0]) / math.log(2.0)
    assert slope == pytest.approx(W.K_MPA, abs=1e-5)
    assert ph[0] == pytest.approx(-(1e-3) ** 8 / (1 + (1e-3) ** 7), rel=1e-14)


# ------------------------------------------ R10: the ansatz at hand points
@pytest.mark.parametrize("theta,x,re,im", [
    ((1, 0, 0, 0, 0, 0, 0, 0), 1.0, 0.5, 0.0),              # x/(1+x^4)
    ((0, 2, 0, 0, 0, 0, 0, 0), 2.0, 8.0 / 17.0, 0.0),       # 2 x^2/(1+x^4)
    ((1, 1, 1, 1, 0, 0, 0, 0), 1.0, 2.0, 0.0),              # (x+x^2+x^3+x^4)/2
    ((0, 0, 0, 0, 0, 0, 0, 3), 0.5, 0.0, 3.0 / 17.0),       # 3 x^4/(1+x^4)
    ((0, 0, 0, 0, 4, 0, -1, 0), 2.0, 0.0, 0.0),             # (4x - x^3)/(1+x^4)
    ((0, 0, 2, 0, 1, 0, 0, 0), 3.0, 54.0 / 82.0, 3.0 / 82.0),
])
def test_ansatz_at_hand_computed_points(theta, x, re, im):
    """f(x) = [sum_p th_p x^p + i sum_p th_{4+p} x^p] / (1 + x^4) applied as
    phase k0 n2 I_a dz Re f and log-amplitude -k0 n2 I_a dz Im f; the
    values are fractions worked out by hand."""
    inst = _inst(terms=W.TERM_ANSATZ, theta=theta)
    scr = M.Screen.of(inst)
    kn_ia = scr.k0 * scr.n2 * scr.dz * W.I_A
    ph, _ = scr.phase(np.array([x * W.I_A]))
    la, _ = scr.log_amp(np.array([x * W.I_A]))
    assert ph[0] == pytest.approx(kn_ia * re, rel=1e-14, abs=1e-300)
    assert la[0] == pytest.approx(-kn_ia * im, rel=1e-14, abs=1e-300)
