"""Forward march, nonlinear screen and discrete adjoint, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The stationary NLSE (Math and Equations, Eq. (1), (3), (9)) is integrated by
the split-step method the paper builds on: each z step applies diffraction
exactly in Fourier space and then a pointwise nonlinear screen (Lie
splitting, diffraction first).  Written here in the propagation convention
dU/dz = (i/2k0) Lap U + i k0 dn(I) U - alpha(I)/2 U, the complex conjugate of
the paper's e^{i omega t} form; intensities are the same in both.

Screen terms (all functions of I = |V|^2 in W/m^2, x = I / I_a):

* Kerr (Eq. (1), eps_k |U|^2):       phase k0 n2 I dz
* plasma (Eq. (3), eps_m term), saturating reading:
                                     phase -k0 n2 I_a dz x^K / (1 + x^(K-1))
* multiphoton absorption (Eq. (3), alpha_m term), dissipative reading, exact
  pointwise solution of dI/dz = -beta_K I^K over one step:
                                     amplitude (1 + (K-1) beta_K I^(K-1) dz)^(-1/(2(K-1)))
* ansatz f_theta (stand-in for the effective lens of Eq. (6), (9)):
  f = [sum_p th_p x^p + i sum_p th_{4+p} x^p] / (1 + x^4), applied as
                                     exp(i k0 n2 I_a dz f)
* turbulence (Eq. (9), eps_t): a precomputed phase plane on screen steps.
"""
from __future__ import annotations

import contextlib
import dataclasses
import math
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

# The 2-D transforms the march uses (numpy's, single-threaded).  fft_workers
# swaps in scipy.fft with a thread count for timing the CPU baseline only:
# the same transform, the march unchanged.
_FFT = {"fft2": np.fft.fft2, "ifft2": np.fft.ifft2}


@contextlib.contextmanager
def fft_workers(workers: int):
    """Run the oracle's 2-D FFTs through scipy.fft with `workers` threads."""
    import scipy.fft as sf
    saved = dict(_FFT)
    _FFT["fft2"] = lambda a: sf.fft2(a, workers=workers)
    _FFT["ifft2"] = lambda a: sf.ifft2(a, workers=workers)
    try:
        yield
    finally:
        _FFT.update(saved)


KERR, MPA, PLASMA, ANSATZ, TURB = 1, 2, 4, 8, 16


# ------------------------------------------------------------- diffraction
def wavenumbers(n: int, length: float) -> np.ndarray:
    """Angular spatial frequencies of an n-point periodic grid of side L."""
    return 2.0 * math.pi * np.fft.fftfreq(n, d=length / n)


def propagator(n: int, length: float, dz: float, k0: float) -> np.ndarray:
    """Full 2-D diffraction factor exp(-i (kx^2 + ky^2) dz / 2k0), [ky, kx].

    The paraxial operator (Laplacian over 2k0, Eq. (1)) is diagonal in
    Fourier space; this is its exact exponential over one step.
    """
    k = wavenumbers(n, length)
    k2 = k[None, :] ** 2 + k[:, None] ** 2
    return np.exp(-1j * k2 * dz / (2.0 * k0))


def diffract(u: np.ndarray, prop: np.ndarray) -> np.ndarray:
    """One exact diffraction step: F^-1 [P . F u]."""
    return _FFT["ifft2"](prop * _FFT["fft2"](u))


def diffract_adjoint(lam: np.ndarray, prop: np.ndarray) -> np.ndarray:
    """Hermitian adjoint of ``diffract``: F^-1 [conj(P) . F lam]."""
    return _FFT["ifft2"](np.conj(prop) * _FFT["fft2"](lam))


# ------------------------------------------------------------------ screen
@dataclasses.dataclass
class Screen:
    """Pointwise nonlinear screen E(I) = A(I) exp(i Phi(I)) of one step."""

    k0: float
    n2: float
    i_ref: float
    order: int
    beta: float
    dz: float
    terms: int
    theta: np.ndarray

    @classmethod
    def of(cls, inst, theta: Optional[Sequence[float]] = None) -> "Screen":
        m = inst.medium
        th = theta if theta is not None else (inst.theta or (0.0,) * 8)
        return cls(k0=2.0 * math.pi / m.wavelength, n2=m.n2, i_ref=m.i_ref,
                   order=m.mpa_order, beta=m.beta_k, dz=inst.dz,
                   terms=m.terms, theta=np.asarray(th, dtype=np.float64))

    # f_theta and its x-derivative
    def _ansatz(self, x):
        den = 1.0 + x ** 4
        re = sum(self.theta[p - 1] * x ** p for p in range(1, 5)) / den
        im = sum(self.theta[3 + p] * x ** p for p in range(1, 5)) / den
        dg_re = sum(p * self.theta[p - 1] * x ** (p - 1) for p in range(1, 5))
        dg_im = sum(p * self.theta[3 + p] * x ** (p - 1) for p in range(1, 5))
        dden = 4.0 * x ** 3
        d_re = dg_re / den - re * dden / den
        d_im = dg_im / den - im * dden / den
        return re, im, d_re, d_im

    def phase(self, i):
        """Phi(I) and dPhi/dI."""
        ph = np.zeros_like(i)
        dph = np.zeros_like(i)
        kn = self.k0 * self.n2 * self.dz
        x = i / self.i_ref
        K = self.order
        if self.terms & KERR:
            ph = ph + kn * i
            dph = dph + kn
        if self.terms & PLASMA:
            s = x ** (K - 1)
            ph = ph - kn * self.i_ref * x ** K / (1.0 + s)
            dph = dph - kn * s * (K + s) / (1.0 + s) ** 2
        if self.terms & ANSATZ:
            re, _, d_re, _ = self._ansatz(x)
            ph = ph + kn * self.i_ref * re
            dph = dph + kn * d_re
        return ph, dph

    def log_amp(self, i):
        """ln A(I) and d ln A / dI."""
        la = np.zeros_like(i)
        dla = np.zeros_like(i)
        K = self.order
        if self.terms & MPA:
            q = 1.0 + (K - 1) * self.beta * i ** (K - 1) * self.dz
            la = la - np.log(q) / (2.0 * (K - 1))
            dla = dla - (K - 1) * self.beta * i ** (K - 2) * self.dz / (2.0 * q)
        if self.terms & ANSATZ:
            kn = self.k0 * self.n2 * self.dz
            x = i / self.i_ref
            _, im, _, d_im = self._ansatz(x)
            la = la - kn * self.i_ref * im
            dla = dla - kn * d_im
        return la, dla

    def factor(self, i):
        ph, _ = self.phase(i)
        la, _ = self.log_amp(i)
        return np.exp(la + 1j * ph)

    def dfactor(self, i):
        """E(I) and dE/dI."""
        ph, dph = self.phase(i)
        la, dla = self.log_amp(i)
        e = np.exp(la + 1j * ph)
        return e, e * (dla + 1j * dph)

    def theta_basis(self, i):
        """d(ln E)/d theta_p for p = 1..8 (Eq. (9) ansatz term, linear in th)."""
        kn = self.k0 * self.n2 * self.dz
        x = i / self.i_ref
        den = 1.0 + x ** 4
        out = []
        for p in range(1, 5):
            out.append(1j * kn * self.i_ref * x ** p / den)
        for p in range(1, 5):
            out.append(-kn * self.i_ref * x ** p / den)
        return out


def apply_screen(v: np.ndarray, scr: Screen,
                 phi_t: Optional[np.ndarray] = None) -> np.ndarray:
    u = v * scr.factor(np.abs(v) ** 2)
    if phi_t is not None:
        u = u * np.exp(1j * phi_t)
    return u


# ------------------------------------------------------------------- march
@dataclasses.dataclass
class MarchResult:
    field: np.ndarray            # U_N, complex128 [y, x]
    power: np.ndarray            # sum |U_{n+1}|^2 dx^2 after each step [W]
    peak: np.ndarray             # max |U_{n+1}|^2 after each step [W/m^2]
    pre_screen: Optional[List[np.ndarray]] = None   # V_n of every step


def march(u0: np.ndarray, inst, n_steps: Optional[int] = None,
          theta: Optional[Sequence[float]] = None,
          screens: Optional[Dict[int, np.ndarray]] = None,
          keep_pre_screen: bool = False, strang: bool = False) -> MarchResult:
    """Split-step march: for each step V = F^-1 P F U, U = V E(|V|^2) T
    (Lie, diffraction first).  With strang=True each step is symmetric:
    V = F^-1 P_h F U, W = V E(|V|^2) T, U = F^-1 P_h F W with P_h the
    half-step propagator (Strang splitting, second order in dz)."""
    n_steps = inst.n_steps if n_steps is None else n_steps
    k0 = 2.0 * math.pi / inst.medium.wavelength
    if strang:
        half = propagator(inst.n, inst.length, inst.dz / 2, k0)
        return _march_strang(u0, inst, n_steps, theta, screens, half)
    prop = propagator(inst.n, inst.length, inst.dz, k0)
    scr = Screen.of(inst, theta)
    turb = screens if (inst.medium.terms & TURB) else None
    dx2 = inst.dx ** 2
    u = np.array(u0, dtype=np.complex128)
    pw = np.empty(n_steps)
    pk = np.empty(n_steps)
    hist = [] if keep_pre_screen else None
    for n in range(n_steps):
        v = diffract(u, prop)
        if hist is not None:
            hist.append(v)
        phi = turb.get(n) if turb else None
        u = apply_screen(v, scr, phi)
        inten = np.abs(u) ** 2
        pw[n] = inten.sum() * dx2
        pk[n] = inten.max()
    return MarchResult(u, pw, pk, hist)


def _march_strang(u0, inst, n_steps, theta, screens, half) -> MarchResult:
    scr = Screen.of(inst, theta)
    turb = screens if (inst.medium.terms & TURB) else None
    dx2 = inst.dx ** 2
    u = np.array(u0, dtype=np.complex128)
    pw = np.empty(n_steps)
    pk = np.empty(n_steps)
    for n in range(n_steps):
        v = diffract(u, half)
        phi = turb.get(n) if turb else None
        u = diffract(apply_screen(v, scr, phi), half)
        inten = np.abs(u) ** 2
        pw[n] = inten.sum() * dx2
        pk[n] = inten.max()
    return MarchResult(u, pw, pk, None)


# ------------------------------------------------------------ loss, adjoint
def block_mean(w: np.ndarray, b: int) -> np.ndarray:
    n = w.shape[0] // b
    return w.reshape(n, b, n, b).mean(axis=(1, 3))


def fluence_loss(u: np.ndarray, target: np.ndarray):
    """L = sum (|U|^2 - w)^2 / sum w^2 and its cotangent G = dL/dRe + i dL/dIm."""
    inten = np.abs(u) ** 2
    den = float(np.sum(target ** 2))
    diff = inten - target
    loss = float(np.sum(diff ** 2)) / den
    g = 4.0 * diff * u / den
    return loss, g


def gradient(u0: np.ndarray, inst, n_steps: Optional[int] = None,
             theta: Optional[Sequence[float]] = None,
             screens: Optional[Dict[int, np.ndarray]] = None,
             cotangent: Optional[Callable] = None, strang: bool = False):
    """Exact discrete adjoint of ``march``.

    ``cotangent(U_N) -> (loss, G_N)`` gives the loss and G = dL/dRe U_N +
    i dL/dIm U_N.  Returns (loss, G w.r.t. U0, dL/dtheta).

    Backward through one step, with lam the cotangent of U_{n+1}:
      lam <- conj(T_n) lam                       (turbulence phase)
      dL/dth_p += Re(conj(lam) U' dlnE/dth_p)    (U' = V E, linear in th)
      lam_V = lam conj(E + I E') + conj(lam) V^2 E'   (E' = dE/dI)
      lam <- F^-1 conj(P) F lam_V                (adjoint diffraction)
    With strang=True the step is U' = P_h (V E T), V = P_h U, so the adjoint
    half-step diffraction comes before and after the same screen adjoint.
    """
    n_steps = inst.n_steps if n_steps is None else n_steps
    k0 = 2.0 * math.pi / inst.medium.wavelength
    scr = Screen.of(inst, theta)
    turb = screens if (inst.medium.terms & TURB) else None
    if strang:
        prop = propagator(inst.n, inst.length, inst.dz / 2, k0)
        u = np.array(u0, dtype=np.complex128)
        pre = []
        for n in range(n_steps):
            v = diffract(u, prop)
            pre.append(v)
            u = diffract(apply_screen(v, scr, turb.get(n) if turb else None), prop)
        loss, lam = cotangent(u)
    else:
        prop = propagator(inst.n, inst.length, inst.dz, k0)
        res = march(u0, inst, n_steps, theta, screens, keep_pre_screen=True)
        pre = res.pre_screen
        loss, lam = cotangent(res.field)
    g_theta = np.zeros(8)
    for n in reversed(range(n_steps)):
        if strang:
            lam = diffract_adjoint(lam, prop)
        v = pre[n]
        phi = turb.get(n) if turb else None
        if phi is not None:
            lam = lam * np.exp(-1j * phi)
        inten = np.abs(v) ** 2
        e, de = scr.dfactor(inten)
        if scr.terms & ANSATZ:
            up = v * e
            for p, basis in enumerate(scr.theta_basis(inten)):
                g_theta[p] += float(np.sum(np.real(np.conj(lam) * up * basis)))
        lam_v = lam * np.conj(e + inten * de) + np.conj(lam) * v * v * de
        lam = diffract_adjoint(lam_v, prop)
    return loss, lam, g_theta


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
