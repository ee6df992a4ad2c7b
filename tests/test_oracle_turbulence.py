"""Pins of the oracle's turbulence-screen generator."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import turbulence as T

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        ctr = [np.array([v], dtype=np.uint64) for v in r[:4]]
        out = T.philox4x32_10(ctr, (r[4], r[5]))
        assert [int(o[0]) for o in out] == r[6:10]


def test_box_muller_gives_independent_unit_normals():
    ctr = np.arange(200000, dtype=np.uint64)
    z = np.zeros_like(ctr)
    o = T.philox4x32_10((ctr, z, z, z), (12345, 678))
    z0, z1 = T.box_muller(T.uniform_open(o[0]), T.uniform_open(o[1]))
    for s in (z0, z1):
        assert stats.kstest(s, "norm").pvalue > 1e-3
        assert abs(s.mean()) < 0.01 and abs(s.var() - 1) < 0.01
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.01


def test_screen_matches_brute_force_inverse_dft():
    n, length = 8, 0.05
    amp = T.kolmogorov_amplitude(n, length, 0.1)
    re, im = T.screen_pair(n, length, amp, 99, 2)
    c = T.white_noise(n, 99, 2) * amp
    phi = np.zeros((n, n), complex)
    for y in range(n):
        for x in range(n):
            for ky in range(n):
                for kx in range(n):
                    phi[y, x] += c[ky, kx] * np.exp(2j * math.pi * (kx * x + ky * y) / n)
    assert np.max(np.abs(re - phi.real)) < 1e-12 * np.abs(phi).max()
    assert np.max(np.abs(im - phi.imag)) < 1e-12 * np.abs(phi).max()


def test_screen_parseval_per_draw():
    n, length = 64, 0.06
    amp = T.kolmogorov_amplitude(n, length, 0.05)
    re, im = T.screen_pair(n, length, amp, 5, 0)
    spec = T.white_noise(n, 5, 0) * amp
    lhs = np.sum(re ** 2 + im ** 2)
    rhs = n * n * np.sum(np.abs(spec) ** 2)
    assert abs(lhs / rhs - 1) < 1e-12


def _discrete_structure(n, length, r0, lags):
    """Exact expectation of the FFT screen's structure function along x:
    D(r) = 2 sum_k Phi(kappa) dkappa^2 (1 - cos(kx r))."""
    amp2 = T.kolmogorov_amplitude(n, length, r0) ** 2
    k = 2 * math.pi * np.fft.fftfreq(n, d=length / n)
    dx = length / n
    return np.array([2 * np.sum(amp2 * (1 - np.cos(k[None, :] * lag * dx)))
                     for lag in lags])


def test_screen_statistics_match_spectrum():
    """Sample structure function of 800 generated screens against its exact
    expectation for the discrete spectrum (pins filter scaling and noise).
    The few lowest modes dominate the larger lags, so fewer screens leave a
    sampling scatter of several per cent."""
    n, length, r0 = 64, 0.06, 0.01
    amp = T.kolmogorov_amplitude(n, length, r0)
    lags = np.arange(1, 9)
    acc = np.zeros(len(lags))
    for p in range(400):
        re, im = T.screen_pair(n, length, amp, 2024, p)
        acc += T.structure_function(re, 8) + T.structure_function(im, 8)
    acc /= 800
    want = _discrete_structure(n, length, r0, lags)
    assert np.all(np.abs(acc / want - 1) < 0.02)


def test_kolmogorov_constant_against_structure_law():
    """The discrete spectrum reproduces the Kolmogorov law
    D(r) = 6.88 (r/r0)^(5/3).  An FFT screen has no power below 1/L or above
    the Nyquist frequency, so its D(r) falls short of the law by a known
    10-25 % on a wide grid (never above it); a wrong 2-pi convention in the
    spectrum constant is off by a factor of 25."""
    n, length, r0 = 4096, 40.0, 0.05
    lags = np.array([2, 4, 8, 16])
    got = _discrete_structure(n, length, r0, lags)
    want = 6.88 * (lags * length / n / r0) ** (5 / 3)
    ratio = got / want
    assert np.all((ratio > 0.78) & (ratio < 1.0))


def test_fried_parameter_textbook_value():
    """r0 = (0.423 k^2 Cn^2 dz)^(-3/5): 800 nm, Cn^2 = 1e-14, 10 m -> ~0.56 m."""
    k0 = 2 * math.pi / 800e-9
    assert abs(T.fried_parameter(k0, 1e-15, 10.0) / 2.2386 - 1) < 1e-3
    assert abs(T.fried_parameter(k0, 1e-14, 10.0) / 0.56231 - 1) < 1e-3


def test_screen_schedule_follows_slab_midplanes():
    """Screen s sits at (s - 1/2) dz_s and follows the step reaching it:
    10 m slabs with dz = 0.1 m give steps 49, 149, ...; exact ties
    (z_s/dz = 1.5, 4.5) round up."""
    import workloads as W
    c3 = W.config3(2)[0]
    assert c3.screen_steps()[:3] == [49, 149, 249]
    tie = W.Instance(n=64, length=0.01, dz=0.01, n_steps=9, medium=W.Medium(),
                     w0=1e-3, power=1.0, sigma=0.0, seed=0, cn2=1e-13,
                     screen_dz=0.03, n_screens=3)
    tie.medium.terms = W.TERM_TURB
    assert tie.screen_steps() == [1, 4, 7]
    assert sorted(T.instance_screens(tie)) == [1, 4, 7]


def test_step_spectrum_screens_are_band_limited():
    """Eq. (10) low-pass step: the screens' own spectrum c amp vanishes
    outside 0 < kappa <= k_h (to rounding), and <phi^2> = tau x (number of
    modes in the band) for both screens of a pair."""
    n, length, tau = 64, 0.05, 2.5e-3
    k_h = 2 * math.pi / length * 6.5
    amp = T.step_amplitude(n, length, tau, k_h)
    band = amp > 0
    assert band.sum() == sum(1 for mx in range(-32, 32) for my in range(-32, 32)
                             if 0 < mx * mx + my * my <= 6.5 ** 2)
    acc = []
    for pair in range(40):
        re, im = T.screen_pair(n, length, amp, 99, pair)
        spec = np.fft.fft2(re + 1j * im) / (n * n)
        assert np.max(np.abs(spec[~band])) < 1e-13 * np.max(np.abs(spec))
        acc += [np.mean(re ** 2), np.mean(im ** 2)]
    want = tau * band.sum()
    assert abs(np.mean(acc) / want - 1) < 0.05


def _expected_d(modes, lag_m):
    """Exact expectation of the structure function along x of Re or Im of
    sum c a exp(2 pi i f.x): each mode adds 2 a^2 (1 - cos(2 pi fx r))."""
    return sum(2 * a * a * (1 - math.cos(2 * math.pi * fx * lag_m)) for _, _, fx, _, a in modes)


def _open_structure(phi, max_lag):
    """Structure function from the pairs inside the window only (subharmonic
    modes are not periodic on it)."""
    return np.array([0.5 * (np.mean((phi[:, lag:] - phi[:, :-lag]) ** 2)
                            + np.mean((phi[lag:, :] - phi[:-lag, :]) ** 2))
                     for lag in range(1, max_lag + 1)])


def test_subharmonic_screens_match_their_expected_structure_function():
    """Sampled structure function of the low-frequency part of 6000 screens
    (3000 pairs) against its exact expectation for the mode list (pins the
    synthesis: coefficients, frequencies on the cell-centred grid, the use of
    the amplitudes).  Few modes carry the variance: over seeds the sample
    mean scatters by about 1 % at this count (3 % at 600 pairs)."""
    n, length, r0 = 32, 1.0, 0.05
    modes = T.subharmonic_modes(length, 3, T.kolmogorov_density(r0))
    lags = np.arange(1, 17)
    acc = np.zeros(len(lags))
    for p in range(3000):
        re, im = T.subharmonic_pair(n, length, modes, 123, p)
        assert abs(re.mean()) < 1e-12 * np.abs(re).max() and abs(im.mean()) < 1e-12 * np.abs(im).max()
        acc += _open_structure(re, 16) + _open_structure(im, 16)
    acc /= 6000
    want = np.array([_expected_d(modes, lag * length / n) for lag in lags])
    assert np.all(np.abs(acc / want - 1) < 0.04), acc / want


def test_subharmonics_close_the_low_frequency_deficit():
    """An FFT screen lacks the power below 1/L, so its D(r) falls far short
    of the Kolmogorov law 6.88 (r/r0)^(5/3) at large r; each subharmonic
    level adds power below the previous one and raises D at every lag, never
    past the law.  Three levels leave the known residual deficit of the
    method: D reaches 0.72-0.83 of the law at L/8 and 0.66-0.78 at L/4 (from
    0.47 and 0.33).  Amplitudes half as large, a level index shifted by one
    or the angular-frequency constant leave these bands."""
    n, length, r0 = 256, 1.0, 0.05
    lags_m = np.array([1, 4, 16, 32, 64, 128]) * length / n
    law = 6.88 * (lags_m / r0) ** (5 / 3)
    fft = _discrete_structure(n, length, r0, np.array([1, 4, 16, 32, 64, 128]))
    dens = T.kolmogorov_density(r0)
    prev = fft / law
    for levels in range(1, 6):
        modes = T.subharmonic_modes(length, levels, dens)
        ratio = (fft + np.array([_expected_d(modes, r) for r in lags_m])) / law
        assert np.all(ratio > prev) and np.all(ratio < 1.0)
        prev = ratio
        if levels == 3:
            assert 0.72 < ratio[3] < 0.83 and 0.66 < ratio[4] < 0.78, ratio
    assert fft[3] / law[3] < 0.5 and fft[4] / law[4] < 0.35


def test_subharmonic_modes_of_the_step_spectrum():
    """The step spectrum as a density is tau per FFT cell, so a subharmonic
    cell of level p carries sqrt(tau) / 3^p, and only inside the band."""
    length, tau = 0.5, 3e-3
    k_h = 2 * math.pi / (3 * length) * 1.2     # above level 1's edge cells, below its corners
    modes = T.subharmonic_modes(length, 2, T.step_density(length, tau, k_h))
    for p, q, fx, fy, a in modes:
        inside = (2 * math.pi) ** 2 * (fx * fx + fy * fy) <= k_h * k_h
        want = math.sqrt(tau) / 3 ** p if inside else 0.0
        assert abs(a - want) <= 1e-15 * math.sqrt(tau)
    assert sum(a == 0 for *_, a in modes) == 4   # the 4 corner cells of level 1


def test_instance_screens_with_subharmonics_add_the_low_part():
    import dataclasses
    import workloads as W
    inst = dataclasses.replace([b for b in W.config3() if b.n == 256][0], n=64)
    base = T.instance_screens(inst)
    same = T.instance_screens(inst, subharmonics=0)
    more = T.instance_screens(inst, subharmonics=3)
    k0 = 2 * math.pi / inst.medium.wavelength
    modes = T.subharmonic_modes(inst.length, 3,
                                T.kolmogorov_density(T.fried_parameter(k0, inst.cn2, inst.screen_dz)))
    lre, lim = T.subharmonic_pair(inst.n, inst.length, modes, inst.seed, 0)
    steps = sorted(base)
    assert all(np.array_equal(base[s], same[s]) for s in steps)
    assert np.allclose(more[steps[0]] - base[steps[0]], lre, atol=1e-12, rtol=0)
    assert np.allclose(more[steps[1]] - base[steps[1]], lim, atol=1e-12, rtol=0)


def _ring(q2):
    """Brute-force count of integer modes with 0 < mx^2 + my^2 <= q2."""
    r = int(math.isqrt(int(q2))) + 1
    return sum(1 for mx in range(-r, r + 1) for my in range(-r, r + 1)
               if 0 < mx * mx + my * my <= q2)


@pytest.mark.parametrize("length", [0.06, 0.05, 8e-3, 0.12, 1.0])
def test_step_band_edge_is_decided_on_integer_modes(length):
    """Eq. (10) band, low-pass reading: a k_h placed on the |m| = 5 ring
    (k_h = 2 pi 5 / L, formed the way a caller would) keeps all 12 modes of
    that ring (m^2 = 25: (+-5, 0), (0, +-5), (+-3, +-4), (+-4, +-3)) for any
    window; one part in 1e9 less drops them.  The decision is on integers,
    so it cannot depend on how a wavenumber was rounded."""
    n = 64
    val = 1.0 / (n * (length / n))
    for k_h in (2.0 * math.pi * (5 * val), 2.0 * math.pi * 5 / length):
        amp = T.step_amplitude(n, length, 1e-3, k_h)
        assert int((amp > 0).sum()) == _ring(25) == 80
        below = T.step_amplitude(n, length, 1e-3, k_h * (1 - 1e-9))
        assert int((below > 0).sum()) == _ring(24) == 80 - 12
    m = T.mode_indices(n)
    assert m[0] == 0 and m[5] == 5 and m[-5] == -5 and m[n // 2] == n // 2


def test_band_radius_in_mode_units():
    """q2 = (k_h L / 2 pi)^2 up to the 2^-40 slack."""
    assert T.band_q2(2.0, 2 * math.pi * 3 / 2.0) == pytest.approx(9.0, rel=1e-12)
    assert 9.0 <= T.band_q2(2.0, 2 * math.pi * 3 / 2.0) < 9.0 * (1 + 2e-12)
    assert T.band_q2(0.5, 2 * math.pi) == pytest.approx(0.25, rel=1e-12)


def test_screens_closer_than_a_step_are_refused():
    """A screen spacing below dz would put two screens on one step (or one
    before the first step): refused rather than silently merged."""
    import workloads as W
    inst = W.Instance(n=16, length=0.01, dz=0.1, n_steps=9, medium=W.Medium(terms=W.TERM_TURB),
                      w0=1e-3, power=1.0, sigma=0.0, seed=0, cn2=1e-14,
                      screen_dz=0.05, n_screens=4)
    with pytest.raises(ValueError):
        T.instance_screens(inst)
    # at screen_dz = dz every screen has its own step, starting at step 0
    inst.screen_dz = 0.1
    assert sorted(T.instance_screens(inst)) == [0, 1, 2, 3]
