"""Random turbulence phase screens (Eq. (9) eps_t, Eq. (10)), FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper builds its turbulent screen by the spectral method: complex white
noise is shaped by the square root of a phase spectrum and inverse Fourier
transformed.  Eq. (10) models the spectrum as a step; the workloads use the
Kolmogorov phase spectrum with the plane-wave Fried parameter of a slab of
thickness dz_s, r0 = (0.423 k0^2 Cn^2 dz_s)^(-3/5) (textbook FFT phase-screen
method); the step spectrum is available as an option.

Normalisation: with spatial frequency f in cycles/m the phase spectrum is
Phi(f) = 0.023 r0^(-5/3) f^(-11/3) and each FFT sample carries
sqrt(Phi(f)) df, df = 1/L.  (Written with angular frequency kappa = 2 pi f
and dkappa = 2 pi / L the constant is 0.023 (2 pi)^(5/3) = 0.49; using 0.023
with kappa would make the structure function 25 times too small.)  This is
what reproduces D(r) = 6.88 (r/r0)^(5/3).

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written here from its definition:
ten rounds of two 32x32->64 multiplies with a Weyl-sequence key schedule.
Counter = (column, row, pair index, 0), key = (seed low word, seed high word).
Two uniforms (u + 1/2) 2^-32 from output words 0 and 1 feed one Box-Muller
transform, giving c = z0 + i z1 for that spectral sample.  One complex draw
gives two screens: the real part (even screen index) and the imaginary part
(odd screen index) of sum_k c_k sqrt(Phi(f_k)) df e^{2 pi i f_k.x}.

An FFT screen has no power below the window's fundamental 1/L.  Optionally
the subharmonic method (Lane, Glindemann and Dainty 1992) adds it back:
levels p = 1..P of 8 modes on a 3 x 3 grid of spacing 1/(3^p L) around
f = 0, each with its own Philox draw (counter word 3 = 1), summed on the
cell-centred grid and made mean-free.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key) -> Tuple[np.ndarray, ...]:
    """Vectorised Philox4x32-10; ``ctr`` is 4 uint32 arrays, ``key`` 2 ints."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in ctr]
    k0 = np.uint64(key[0] & 0xFFFFFFFF)
    k1 = np.uint64(key[1] & 0xFFFFFFFF)
    m0 = np.uint64(PHILOX_M[0])
    m1 = np.uint64(PHILOX_M[1])
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W[0])) & _MASK
            k1 = (k1 + np.uint64(PHILOX_W[1])) & _MASK
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return tuple(v.astype(np.uint32) for v in c)


def uniform_open(u32: np.ndarray) -> np.ndarray:
    """Map a 32-bit word to (0, 1): (u + 1/2) / 2^32."""
    return (u32.astype(np.float64) + 0.5) * 2.0 ** -32


def box_muller(u1: np.ndarray, u2: np.ndarray):
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * math.pi * u2), r * np.sin(2.0 * math.pi * u2)


def white_noise(n: int, seed: int, pair: int) -> np.ndarray:
    """Complex unit-variance-per-component noise c[row, col] of one draw."""
    col = np.tile(np.arange(n, dtype=np.uint64), n)
    row = np.repeat(np.arange(n, dtype=np.uint64), n)
    zero = np.zeros(n * n, dtype=np.uint64)
    pr = np.full(n * n, pair, dtype=np.uint64)
    o = philox4x32_10((col, row, pr, zero), (seed & 0xFFFFFFFF, seed >> 32))
    z0, z1 = box_muller(uniform_open(o[0]), uniform_open(o[1]))
    return (z0 + 1j * z1).reshape(n, n)


def fried_parameter(k0: float, cn2: float, dz_s: float) -> float:
    return (0.423 * k0 ** 2 * cn2 * dz_s) ** (-3.0 / 5.0)


def kolmogorov_amplitude(n: int, length: float, r0: float) -> np.ndarray:
    """sqrt(Phi(f)) df on the FFT grid [row, col]; zero at f = 0."""
    f = np.fft.fftfreq(n, d=length / n)
    fr = np.sqrt(f[None, :] ** 2 + f[:, None] ** 2)
    psd = np.zeros_like(fr)
    nz = fr > 0
    psd[nz] = 0.023 * r0 ** (-5.0 / 3.0) * fr[nz] ** (-11.0 / 3.0)
    return np.sqrt(psd) / length


def band_q2(length: float, k_h: float) -> float:
    """Squared radius of the Eq. (10) band in mode-index units, with a
    relative slack of 2^-40: q2 = (k_h L / 2 pi)^2 (1 + 2^-40).  A mode
    (mx, my) of spatial frequency (mx, my)/L has kappa = 2 pi |m| / L, so
    kappa <= k_h reads |m|^2 <= (k_h L / 2 pi)^2; the slack keeps a ring
    that k_h was placed on (k_h = 2 pi M / L) inside whatever the rounding
    of that product, so the edge is decided on integers."""
    q = k_h * length / (2.0 * math.pi)
    return q * q * (1.0 + 2.0 ** -40)


def mode_indices(n: int) -> np.ndarray:
    """Signed integer mode index m of each FFT sample (fftfreq order)."""
    m = np.arange(n, dtype=np.int64)
    return np.where(m <= n // 2, m, m - n)


def step_amplitude(n: int, length: float, tau: float, k_h: float) -> np.ndarray:
    """Eq. (10) read as a low-pass step: sqrt(tau) for 0 < kappa <= k_h.
    The band is decided on the integer mode indices, 0 < mx^2 + my^2 <= q2
    (``band_q2``), so no rounding of a wavenumber enters the decision."""
    m = mode_indices(n)
    m2 = m[None, :] ** 2 + m[:, None] ** 2
    q2 = band_q2(length, k_h)
    return np.where((m2 > 0) & (m2 <= q2), math.sqrt(tau), 0.0)


def screen_pair(n: int, length: float, amp: np.ndarray, seed: int,
                pair: int) -> Tuple[np.ndarray, np.ndarray]:
    """Two phase screens [rad] from one draw: phi = N^2 IFFT2(c amp)."""
    spec = white_noise(n, seed, pair) * amp
    phi = np.fft.ifft2(spec) * (n * n)
    return phi.real.copy(), phi.imag.copy()


def kolmogorov_density(r0: float):
    """Phase spectral density Phi(fx, fy) = 0.023 r0^(-5/3) f^(-11/3) [rad^2 m^2]
    (called as dens(fx, fy, (p, mx, my)); the mode indices are not used)."""
    return lambda fx, fy, idx=None: (0.023 * r0 ** (-5.0 / 3.0)
                                     * math.hypot(fx, fy) ** (-11.0 / 3.0))


def step_density(length: float, tau: float, k_h: float):
    """The Eq. (10) step as a density: tau per FFT cell of area 1/L^2, i.e.
    tau L^2, inside the band.  Subharmonic modes sit at f = (mx, my)/(3^p L),
    so kappa <= k_h reads mx^2 + my^2 <= 9^p q2 with the integer indices
    and the same q2 as the FFT modes (``band_q2``).  Called as
    dens(fx, fy, (p, mx, my))."""
    q2 = band_q2(length, k_h)

    def dens(fx, fy, idx):
        p, mx, my = idx
        return tau * length * length if mx * mx + my * my <= q2 * 9 ** p else 0.0
    return dens


def subharmonic_modes(length: float, levels: int, density):
    """Modes of the subharmonic method (Lane, Glindemann and Dainty, Waves in
    Random Media 2 (1992) 209): at level p = 1..levels the frequency cell
    df_p = 1/(3^p L) is split around f = 0 into a 3 x 3 grid, and each of the
    8 outer cells is one mode f = (mx, my) df_p with amplitude
    sqrt(density(f)) df_p.  Returns (p, q, fx, fy, a) with q = 3 (my + 1) +
    (mx + 1) the cell's index (the centre, q = 4, is skipped)."""
    out = []
    for p in range(1, levels + 1):
        df = 1.0 / (3 ** p * length)
        for q in range(9):
            if q == 4:
                continue
            mx, my = q % 3 - 1, q // 3 - 1
            fx, fy = mx * df, my * df
            out.append((p, q, fx, fy, math.sqrt(density(fx, fy, (p, mx, my))) * df))
    return out


def subharmonic_pair(n: int, length: float, modes, seed: int,
                     pair: int) -> Tuple[np.ndarray, np.ndarray]:
    """Low-frequency part of screen pair `pair`: lo(x, y) = sum c a
    exp(2 pi i (fx x + fy y)) over the modes, on the cell-centred grid, minus
    its mean over the grid; real part for the even screen, imaginary part for
    the odd one.  The coefficient c of mode (p, q) is one Box-Muller draw from
    Philox counter (q, p, pair, 1) (the FFT noise uses counter word 3 = 0)."""
    x = (np.arange(n) + 0.5 - n / 2) * (length / n)
    lo = np.zeros((n, n), dtype=np.complex128)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for p, q, fx, fy, a in modes:
        o = philox4x32_10(([q], [p], [pair], [1]), key)
        z0, z1 = box_muller(uniform_open(o[0]), uniform_open(o[1]))
        c = complex(z0[0], z1[0])
        lo += c * a * np.exp(2j * math.pi * (fx * x[None, :] + fy * x[:, None]))
    lo -= lo.mean()
    return lo.real.copy(), lo.imag.copy()


def instance_screens(inst, step_spectrum=None, subharmonics: int = 0) -> Dict[int, np.ndarray]:
    """Screens of an instance keyed by the step they follow: Kolmogorov, or
    with step_spectrum = (tau, k_h) the Eq. (10) low-pass step; with
    subharmonics = P the low-frequency part of P subharmonic levels of the
    same spectrum is added to every screen."""
    if inst.n_screens <= 0:
        return {}
    if not inst.screen_dz >= inst.dz:
        # closer screens could fall on one step (or before the first)
        raise ValueError("screen spacing %g m is below the step %g m" % (inst.screen_dz, inst.dz))
    if step_spectrum is not None:
        amp = step_amplitude(inst.n, inst.length, *step_spectrum)
        dens = step_density(inst.length, *step_spectrum)
    else:
        k0 = 2.0 * math.pi / inst.medium.wavelength
        r0 = fried_parameter(k0, inst.cn2, inst.screen_dz)
        amp = kolmogorov_amplitude(inst.n, inst.length, r0)
        dens = kolmogorov_density(r0)
    modes = subharmonic_modes(inst.length, subharmonics, dens)
    steps = []
    for s in range(1, inst.n_screens + 1):
        # the step that reaches the slab mid-plane z_s (ties round up)
        steps.append(int(math.floor((s - 0.5) * inst.screen_dz / inst.dz + 0.5)) - 1)
    out = {}
    for p in range((inst.n_screens + 1) // 2):
        re, im = screen_pair(inst.n, inst.length, amp, inst.seed, p)
        if modes:
            lre, lim = subharmonic_pair(inst.n, inst.length, modes, inst.seed, p)
            re, im = re + lre, im + lim
        out[steps[2 * p]] = re
        if 2 * p + 1 < inst.n_screens:
            out[steps[2 * p + 1]] = im
    return out


def structure_function(phi: np.ndarray, max_lag: int) -> np.ndarray:
    """<(phi(x+r) - phi(x))^2> along both axes for lags 1..max_lag (periodic)."""
    out = np.empty(max_lag)
    for lag in range(1, max_lag + 1):
        dx = np.roll(phi, -lag, axis=1) - phi
        dy = np.roll(phi, -lag, axis=0) - phi
        out[lag - 1] = 0.5 * (np.mean(dx ** 2) + np.mean(dy ** 2))
    return out
