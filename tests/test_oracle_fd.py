"""Pins of the oracle's finite-difference reference scheme (Crank-Nicolson
with the nonlinearity at the mean intensity, 5-point Laplacian, periodic).

Pinned by what the discretisation and the mathematics fix: the Laplacian's
plane-wave eigenvalues, the Cayley factor of a linear step, the exact
conservation of power and of the Kerr Hamiltonian by converged steps, the
discrete energy balance with multiphoton absorption, second order in dz and
in dx, and agreement with the split-step march as both are refined (the
cross-validation the paper uses the scheme for).
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd as FD
from oracle import march as M


def _beam(n=64, terms=W.TERM_KERR, **kw):
    base = W.config1()[0]
    return dataclasses.replace(base, n=n, medium=dataclasses.replace(base.medium, terms=terms),
                               **kw)


def _strong(terms, n=64, dz=2.5e-4):
    """Peak intensity 1.1 I_a (1.23 I_a with the noise): multiphoton
    absorption removes ~1 % of the power per step of 0.25 mm, plasma
    defocusing is active, and the fixed point converges (~30 iterations to
    1e-15; at dz = 1 mm its contraction factor nears 1)."""
    w0 = 0.3e-3
    power = 1.1 * W.I_A * math.pi * w0 * w0 / 2
    return W.Instance(n=n, length=2e-3, dz=dz, n_steps=10, medium=W.Medium(terms=terms),
                      w0=w0, power=power, sigma=0.1, seed=5)


def test_laplacian_plane_wave_eigenvalues():
    n, dx = 12, 0.37
    lap = FD.laplacian(n, dx)
    j = np.arange(n)
    for mx, my in [(0, 0), (1, 0), (0, 5), (3, 7), (6, 6), (11, 2)]:
        e = np.exp(2j * math.pi * (mx * j[None, :] + my * j[:, None]) / n).reshape(n * n)
        lam = -(4 / dx ** 2) * (math.sin(math.pi * mx / n) ** 2 + math.sin(math.pi * my / n) ** 2)
        assert np.max(np.abs(lap @ e - lam * e)) < 1e-12 * abs(lam) + 1e-12


def test_laplacian_is_symmetric_negative_semidefinite():
    lap = FD.laplacian(8, 0.1).toarray()
    assert np.array_equal(lap, lap.T)
    ev = np.linalg.eigvalsh(lap)
    assert ev.max() < 1e-9 and abs(ev.max()) < 1e-9 and ev.min() < -1.0


def test_linear_step_multiplies_each_mode_by_its_cayley_factor():
    inst = _beam(n=16, terms=0)
    n, dx = inst.n, inst.dx
    k0 = 2 * math.pi / inst.medium.wavelength
    a = inst.dz / (4 * k0)
    j = np.arange(n)
    st = FD.FDStepper(inst)
    for mx, my in [(1, 0), (2, 3), (8, 8)]:
        e = np.exp(2j * math.pi * (mx * j[None, :] + my * j[:, None]) / n)
        lam = -(4 / dx ** 2) * (math.sin(math.pi * mx / n) ** 2 + math.sin(math.pi * my / n) ** 2)
        got, _, _ = st.step(e, iterations=1)
        want = e * (1 + 1j * a * lam) / (1 - 1j * a * lam)
        assert np.max(np.abs(got - want)) < 1e-13


def test_converged_steps_conserve_power_and_the_kerr_hamiltonian():
    inst = _beam()
    u0 = W.initial_field(inst)
    r = FD.fd_march(u0, inst, 20)
    p0 = float(np.sum(np.abs(u0) ** 2)) * inst.dx ** 2
    assert np.max(np.abs(r.power / p0 - 1)) < 1e-13
    h0, h1 = FD.hamiltonian(u0, inst), FD.hamiltonian(r.field, inst)
    assert abs(h1 / h0 - 1) < 1e-12
    # not trivially constant: the quartic part (and so the gradient part) moves
    q0 = float(np.sum(np.abs(u0) ** 4))
    q1 = float(np.sum(np.abs(r.field) ** 4))
    assert abs(q1 / q0 - 1) > 1e-3


def test_plasma_and_kerr_phases_conserve_power():
    inst = _strong(W.TERM_KERR | W.TERM_PLASMA)
    u0 = W.initial_field(inst)
    r = FD.fd_march(u0, inst, 10)
    p0 = float(np.sum(np.abs(u0) ** 2)) * inst.dx ** 2
    assert max(r.iterations) < 100
    assert np.max(np.abs(r.power / p0 - 1)) < 1e-13


def test_multiphoton_loss_obeys_the_discrete_energy_balance():
    """Converged step: P+ - P = 2 dz dx^2 sum Re G(J) |Ubar|^2 exactly."""
    inst = _strong(W.KPM)
    u = W.initial_field(inst)
    st = FD.FDStepper(inst)
    dx2 = inst.dx ** 2
    for _ in range(5):
        up, k, _ = st.step(u)
        assert k < 100
        ubar = 0.5 * (up + u)
        j = 0.5 * (np.abs(up) ** 2 + np.abs(u) ** 2)
        lhs = (np.sum(np.abs(up) ** 2) - np.sum(np.abs(u) ** 2)) * dx2
        rhs = 2 * inst.dz * dx2 * np.sum(np.real(FD.generator(j, inst)) * np.abs(ubar) ** 2)
        p = np.sum(np.abs(u) ** 2) * dx2
        assert lhs < -1e-4 * p                      # the loss is real
        assert abs(lhs - rhs) < 1e-12 * p
        u = up


def test_fixed_point_iteration_contracts():
    inst = _beam()
    u0 = W.initial_field(inst)
    st = FD.FDStepper(inst)
    ch = [st.step(u0, k)[2] for k in range(1, 7)]
    assert all(b < a / 10 for a, b in zip(ch, ch[1:])), ch


def test_second_order_in_dz():
    inst = _beam(sigma=0.0)
    u0 = W.initial_field(inst)
    z = 40 * inst.dz
    ref = FD.fd_march(u0, dataclasses.replace(inst, dz=z / 640), 640).field
    errs = [np.linalg.norm(FD.fd_march(u0, dataclasses.replace(inst, dz=z / s), s).field - ref)
            for s in (20, 40, 80)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.7 < r1 < 4.3 and 3.7 < r2 < 4.3, (r1, r2)


def test_second_order_in_dx_against_exact_diffraction():
    """Linear diffraction of the Gaussian beam: the 5-point Laplacian's
    error falls 4x per halving of dx (the spectral propagator is exact)."""
    base = _beam(terms=0, sigma=0.0)
    z = 40 * base.dz
    k0 = 2 * math.pi / base.medium.wavelength
    errs = []
    for n in (32, 64, 128):
        inst = dataclasses.replace(base, n=n, dz=z / 40)
        u0 = W.initial_field(inst)
        got = FD.fd_march(u0, inst, 40, iterations=1).field
        errs.append(M.rel_l2(got, M.diffract(u0, M.propagator(n, inst.length, z, k0))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, (r1, r2)


def test_cross_validates_with_the_split_step_march():
    """Kerr beam: finite differences (converged) against the split-step
    march at a fine dz; both discretise the same equation, so their
    difference falls as the FD grid and step are refined together."""
    base = _beam(sigma=0.0)
    z = 40 * base.dz
    diffs = []
    for n, steps in ((32, 40), (64, 80), (128, 160)):
        inst = dataclasses.replace(base, n=n, dz=z / steps)
        u0 = W.initial_field(inst)
        fd = FD.fd_march(u0, inst, steps).field
        ss = M.march(u0, dataclasses.replace(inst, dz=z / 4000), n_steps=4000).field
        diffs.append(M.rel_l2(fd, ss))
    assert 3.5 < diffs[0] / diffs[1] < 4.3 and 3.5 < diffs[1] / diffs[2] < 4.3, diffs
    assert diffs[2] < 5e-4


def test_unsupported_terms_are_refused():
    inst = _beam(terms=W.TERM_KERR | W.TERM_ANSATZ)
    with pytest.raises(ValueError):
        FD.generator(np.ones((4, 4)), inst)
