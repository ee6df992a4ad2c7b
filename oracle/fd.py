"""Semi-implicit conservative finite-difference reference scheme, FP64 CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes its dense reference solutions of Eq. (3) with a
semi-implicit finite-difference scheme that conserves the integrals of
motion (Math and Equations, after Eq. (3)).  The scheme itself is not
printed; the reading here is Crank-Nicolson in z with the nonlinearity taken
at the step's mean intensity (the conservative scheme of Delfour, Fortin and
Payre, J. Comput. Phys. 44 (1981) 277) on the periodic transverse grid with
the 5-point Laplacian Lap_h, in the propagation convention of the march:

    (U+ - U) / dz = (i / 2k0) Lap_h Ubar + G(J) Ubar,    Ubar = (U+ + U) / 2,
    J = (|U+|^2 + |U|^2) / 2,
    G(I) = i k0 n2 [I - I_a x^K / (1 + x^(K-1))] - beta_K I^(K-1) / 2,   x = I / I_a,

G holding the generators of the screen terms that are switched on (Kerr,
saturating plasma, multiphoton absorption: each screen of the split-step
march is the exact solution of dU/dz = G U over one step).  Written for the
mean field, Ubar = (1 - (i dz / 4k0) Lap_h)^-1 [U + (dz/2) G(J) Ubar] with
J = (|2 Ubar - U|^2 + |U|^2) / 2, solved by fixed-point iteration from
Ubar = U; then U+ = 2 Ubar - U.  The linear solve is a sparse LU of the
n^2 x n^2 matrix.

With a real-phase G (no absorption) a converged step conserves sum |U|^2
exactly; for the Kerr term alone it also conserves the discrete Hamiltonian
(1/2k0) <U, -Lap_h U> - (k0 n2 / 2) sum |U|^4.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

KERR, MPA, PLASMA, ANSATZ, TURB = 1, 2, 4, 8, 16


def laplacian(n: int, dx: float) -> sp.csr_matrix:
    """Periodic 5-point Laplacian on the n x n grid, row-major [y, x]."""
    one = sp.identity(n, format="csr")
    d1 = sp.diags([np.ones(n - 1), np.ones(n - 1), [1.0], [1.0]], [1, -1, n - 1, -(n - 1)],
                  shape=(n, n), format="csr")
    lap1 = (d1 - 2.0 * one) / (dx * dx)
    return (sp.kron(one, lap1) + sp.kron(lap1, one)).tocsr()


def generator(intensity: np.ndarray, inst) -> np.ndarray:
    """G(I) of the active terms, complex [1/m]."""
    m = inst.medium
    terms = m.terms
    if terms & (ANSATZ | TURB):
        raise ValueError("the finite-difference reference covers the Kerr, plasma and "
                         "multiphoton terms of Eq. (3) only")
    k0 = 2.0 * math.pi / m.wavelength
    x = intensity / m.i_ref
    g = np.zeros(intensity.shape, dtype=np.complex128)
    if terms & KERR:
        g += 1j * k0 * m.n2 * intensity
    if terms & PLASMA:
        g -= 1j * k0 * m.n2 * m.i_ref * x ** m.mpa_order / (1.0 + x ** (m.mpa_order - 1))
    if terms & MPA:
        g -= 0.5 * m.beta_k * intensity ** (m.mpa_order - 1)
    return g


@dataclasses.dataclass
class FDResult:
    field: np.ndarray           # U_N, complex128 [y, x]
    power: np.ndarray           # sum |U_{n+1}|^2 dx^2 after each step [W]
    peak: np.ndarray            # max |U_{n+1}|^2 after each step [W/m^2]
    iterations: List[int]       # fixed-point iterations of each step
    change: List[float]         # max |Ubar_k - Ubar_{k-1}| / max |Ubar_k| of the last one


class FDStepper:
    """One beam's Crank-Nicolson steps with the LU of 1 - (i dz / 4k0) Lap_h."""

    def __init__(self, inst):
        self.inst = inst
        n = inst.n
        k0 = 2.0 * math.pi / inst.medium.wavelength
        self.a = inst.dz / (4.0 * k0)
        lap = laplacian(n, inst.dx)
        mat = (sp.identity(n * n, format="csc", dtype=np.complex128)
               - 1j * self.a * lap.astype(np.complex128)).tocsc()
        self.lu = spla.splu(mat)

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        n = self.inst.n
        return self.lu.solve(rhs.reshape(n * n)).reshape(n, n)

    def step(self, u: np.ndarray, iterations: Optional[int] = None, tol: float = 1e-15,
             max_iter: int = 500):
        """One step.  iterations = K: exactly K fixed-point iterations (the
        map the GPU computes); None: iterate until the relative change of
        Ubar is below tol (at most max_iter)."""
        half_dz = 0.5 * self.inst.dz
        ubar = u.copy()
        k = 0
        change = math.inf
        while True:
            j = 0.5 * (np.abs(2.0 * ubar - u) ** 2 + np.abs(u) ** 2)
            new = self.solve(u + half_dz * generator(j, self.inst) * ubar)
            change = float(np.max(np.abs(new - ubar)) / np.max(np.abs(new)))
            ubar = new
            k += 1
            if iterations is not None:
                if k >= iterations:
                    break
            elif change <= tol or k >= max_iter:
                break
        return 2.0 * ubar - u, k, change


def fd_march(u0: np.ndarray, inst, n_steps: Optional[int] = None,
             iterations: Optional[int] = None, tol: float = 1e-15) -> FDResult:
    n_steps = inst.n_steps if n_steps is None else n_steps
    st = FDStepper(inst)
    dx2 = inst.dx ** 2
    u = np.array(u0, dtype=np.complex128)
    pw, pk, its, ch = np.empty(n_steps), np.empty(n_steps), [], []
    for s in range(n_steps):
        u, k, c = st.step(u, iterations, tol)
        inten = np.abs(u) ** 2
        pw[s] = inten.sum() * dx2
        pk[s] = inten.max()
        its.append(k)
        ch.append(c)
    return FDResult(u, pw, pk, its, ch)


def hamiltonian(u: np.ndarray, inst) -> float:
    """(1/2k0) <U, -Lap_h U> dx^2 - (k0 n2 / 2) sum |U|^4 dx^2 (Kerr)."""
    k0 = 2.0 * math.pi / inst.medium.wavelength
    n = inst.n
    v = u.reshape(n * n)
    grad = float(np.real(np.vdot(v, -(laplacian(n, inst.dx) @ v))))
    return (grad / (2.0 * k0) - 0.5 * k0 * inst.medium.n2 * float(np.sum(np.abs(u) ** 4))) \
        * inst.dx ** 2
