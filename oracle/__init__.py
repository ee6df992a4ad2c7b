"""FP64 CPU oracle of the split-step (phase-screen) NLSE march.

TEST INFRASTRUCTURE ONLY.  This package is imported by ``tests/``, by the
``smoke()`` check of the entry module and by the CPU-baseline leg of the
benchmark, and by nothing else.  The GPU library never imports, links or
runs it, and it shares no code with the HIP path: it uses numpy's FFT, builds
the full 2-D propagator instead of the separable one, works in SI units
instead of normalised intensity, and draws its own Philox numbers.

Modules
-------
``march``       forward march, nonlinear screen, diagnostics, discrete adjoint
``turbulence``  Philox4x32-10, Box-Muller and the Kolmogorov FFT phase screen

Pinned by the ``-m "not gpu"`` tests (brute-force DFT, Gaussian-beam closed
form, plane-wave closed forms, power conservation, symmetry, convergence
order, Philox known-answer vectors, Parseval and structure-function checks,
finite differences and an independent autodiff of the same map).  The
multifilament march as a whole has no closed form: beyond those pins its
parity is "same discrete map", which is all the GPU tests claim.
"""
from . import march, turbulence  # noqa: F401
