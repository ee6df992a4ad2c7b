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


def _profile_terms(r: np.ndarray, segments):
    """Per segment j: the mask of r on [r_{j-1}, r_j), cos and sin of
    (freq r + phase) there."""
    out = []
    r_lo = 0.0
    for r_hi, amp, freq, phase in segments:
        sel = (r >= r_lo) & (r < r_hi)
        arg = freq * r + phase
        out.append((sel, amp, freq, np.cos(arg), np.sin(arg)))
        r_lo = r_hi
    return out


def lens_vjp(u: np.ndarray, g_out: np.ndarray, length: float, lens: Lens):
    """Vector-Jacobian product of apply_lens at u.

    Cotangents follow G = dL/dRe U + i dL/dIm U, so dL = Re sum conj(G) dU.
    With E = exp(i f(w_dif)), f = f_re + i f_im on the active points:
      dU_out = E dU + U E i f'(w_dif) dw_dif,  dw_dif = Gauss(2 Re(conj(U) dU)),
    and with z = conj(G_out) U E, q_re = -Im z, q_im = -Re z (the factors of
    the real and imaginary parts of f in dL),
      h     = q_re df_re/dw + q_im df_im/dw          (active points)
      G_in  = conj(E) G_out + 2 Gauss(h) U            (Gauss is symmetric)
      dL/dp = sum q_re df_re/dp + q_im df_im/dp       (profile parameters, c1, c2).
    Returns (G_in, grad) with grad = [dL/dc1, dL/dc2, then (a, omega, psi) of
    each real segment, then (b, nu, eta) of each imaginary one].  The
    trimming level, the joining points and l_dif are not differentiated
    (the first two are discontinuities of f)."""
    w = np.abs(u) ** 2
    w_dif = filtered_intensity(w, length, lens.l_dif)
    active = w_dif >= lens.w_l
    arg = np.where(active, w_dif / lens.c1 + lens.c2, 0.0)
    r = np.cbrt(np.maximum(arg, 0.0))
    inside = active & (arg > 0.0)
    f_re, f_im, _ = lens_exponent(u, length, lens)
    e = np.where(active, np.exp(-f_im) * np.exp(1j * f_re), 1.0)
    z = np.conj(g_out) * u * e
    q_re = np.where(active, -z.imag, 0.0)
    q_im = np.where(active, -z.real, 0.0)
    # d(profile)/dr of each part and the per-parameter sums
    dp_dr = np.zeros_like(w)
    grad_seg = []
    for part, q in ((lens.re, q_re), (lens.im, q_im)):
        dpart = np.zeros_like(w)
        for sel, amp, freq, cs, sn in _profile_terms(r, part):
            m = sel & active
            dpart[m] = -amp * freq * sn[m]
            grad_seg += [float(np.sum(q[m] * cs[m])),
                         float(np.sum(q[m] * (-amp * r[m] * sn[m]))),
                         float(np.sum(q[m] * (-amp * sn[m])))]
        dp_dr += q * dpart
    # r = cbrt(w / c1 + c2): dr/dw = 1 / (3 c1 r^2), dr/dc1 = -w / (3 c1^2 r^2),
    # dr/dc2 = 1 / (3 r^2), where the cube root's argument is positive
    inv3r2 = np.where(inside, 1.0 / (3.0 * np.where(inside, r, 1.0) ** 2), 0.0)
    h = dp_dr * inv3r2 / lens.c1
    g_c1 = float(np.sum(dp_dr * inv3r2 * (-w_dif / lens.c1 ** 2)))
    g_c2 = float(np.sum(dp_dr * inv3r2))
    g_in = np.conj(e) * g_out + 2.0 * filtered_intensity(h, length, lens.l_dif) * u
    return g_in, np.array([g_c1, g_c2] + grad_seg)
