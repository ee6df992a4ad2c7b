"""MI355X (gfx950) split-step phase-screen march of the stationary NLSE.

The hot path of Bulygin & Geints (arXiv 2306.15678): the split-step Fourier
march of the (2D+1) nonlinear Schroedinger equation (Math and Equations,
Eq. (1), (3), (9)) with Kerr, multiphoton absorption, saturating plasma,
an ansatz screen and Kolmogorov turbulence screens, its exact discrete
adjoint, and batched uneven beams.  The arithmetic lives in hand-written
HIP kernels behind the C ABI of ``include/ssfm.h`` (``libssfm.so``); this
package is argument marshalling plus a ``torch.autograd.Function``.
"""
from ._lib import (ANSATZ, DEVICE, FP32, FP64, HOST, KERR, MPA, PLASMA, TURB,  # noqa: F401
                   InstanceDesc, SsfmError)
from .march import Propagator, desc_of, make_desc, plan_variants  # noqa: F401
