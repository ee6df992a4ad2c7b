"""The effective-lens screen D_f of the paper (Math and Equations, Eq. (4)-(6)).

Test infrastructure, like the rest of ``oracle/``: plain FP64 numpy, used
only by the tests.

Steps, in the paper's order:
1. Eq. (4): the intensity w = |U|^2 passed through a Fourier-space filter,
   w_dif = F^-1 [exp(-l_dif k^2) F w]  (the filter read as a Gaussian in k,
   k^2 = kx^2 + ky^2 on the march's grid wavenumbers);
2. trimming at the boundary level w_l: the lens field w_lens = w_dif where
   w_dif >= w_l; elsewhere there is no lens;
3. Eq. (5): the distance to the lens centre from the monotone lens field,
   inverting the cubic w_lens = c1 (r^3 - c2): r = cbrt(w_lens / c1 + c2),
   clamped at r >= 0;
4. Eq. (6): the piecewise-cosine profile, real part sum_j a_j cos(omega_j r
   + psi_j) on r_{j-1} <= r < r_j (r_0 = 0) and imaginary part likewise with
   (r_l, b_l, nu_l, eta_l), zero beyond the last joining point;
5. the lens as one screen: U <- U exp(i f_lens) = U exp(-Im f) e^{i Re f}.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass
class Lens:
    l_dif: float                 # [m^2]
    w_l: float                   # [W/m^2]
    c1: float                    # [W/m^2 / m^3]
    c2: float                    # [m^3]
    re: List[Tuple[float, float, float, float]] = field(default_factory=list)  # (r_j, a, omega, psi)
    im: List[Tuple[float, float, float, float]] = field(default_factory=list)  # (r_l, b, nu, eta)


def filtered_intensity(w: np.ndarray, length: float, l_dif: float) -> np.ndarray:
    """Eq. (4): real(F^-1 [exp(-l_dif k^2) F w]) with the 2-D FFT."""
    n = w.shape[0]
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=length / n)
    filt = np.exp(-l_dif * (k[None, :] ** 2 + k[:, None] ** 2))
    return np.real(np.fft.ifft2(filt * np.fft.fft2(w)))


def radius(w_lens: np.ndarray, c1: float, c2: float) -> np.ndarray:
    """Eq. (5) inverted: r with c1 (r^3 - c2) = w_lens, r >= 0."""
    return np.cbrt(np.maximum(w_lens / c1 + c2, 0.0))


def profile(r: np.ndarray, segments) -> np.ndarray:
    """Eq. (6), one part: sum over segments of amp cos(freq r + phase) on
    [r_{j-1}, r_j)."""
    out = np.zeros_like(r, dtype=np.float64)
    r_lo = 0.0
    for r_hi, amp, freq, phase in segments:
        sel = (r >= r_lo) & (r < r_hi)
        out[sel] = amp * np.cos(freq * r[sel] + phase)
        r_lo = r_hi
    return out


def lens_exponent(u: np.ndarray, length: float, lens: Lens):
    """(f_re, f_im, active) of the lens for the field u."""
    w = np.abs(u) ** 2
    w_dif = filtered_intensity(w, length, lens.l_dif)
    active = w_dif >= lens.w_l
    r = radius(np.where(active, w_dif, 0.0), lens.c1, lens.c2)
    f_re = np.where(active, profile(r, lens.re), 0.0)
    f_im = np.where(active, profile(r, lens.im), 0.0)
    return f_re, f_im, active


def apply_lens(u: np.ndarray, length: float, lens: Lens) -> np.ndarray:
    """U exp(i f_lens) where the lens is present, U elsewhere."""
    f_re, f_im, active = lens_exponent(u, length, lens)
    return np.where(active, u * np.exp(-f_im) * np.exp(1j * f_re), u)
