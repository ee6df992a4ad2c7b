"""The allocation-free hot-area count (a fixed device scratch array in the
library, no context) against the context entry point, through the C ABI.

Two calls in a row, the second on a smaller grid (the array keeps the first
call's labels: the second must not see them), each equal to ssfm_hot_areas
on the same array (integer counts: bit-exact), and both against the
oracle's labelling.  The size limit is refused before any device work.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as D

pytestmark = pytest.mark.gpu


def _fluence(n, seed):
    """Seeded speckle-like fluence: smoothed squared complex noise."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    k = np.fft.fftfreq(n)
    filt = np.exp(-(k[None, :] ** 2 + k[:, None] ** 2) / (2 * 0.03 ** 2))
    v = np.fft.ifft2(np.fft.fft2(u) * filt)
    return np.abs(v) ** 2


def test_static_hot_areas_match_the_context_entry_point():
    import torch
    from paper_2306_15678_amd import _lib as L
    from paper_2306_15678_amd.march import Propagator, desc_of, hot_areas_static
    inst = W.scaled(W.config2()[0], 2048, 1)
    p = Propagator([desc_of(inst)], precision=32)
    for n, seed, frac, periodic in ((2048, 1, 0.3, True), (512, 2, 0.2, False)):
        w = _fluence(n, seed)
        thr = frac * float(w.max())
        wd = torch.from_numpy(w).cuda()
        got = hot_areas_static(wd, thr, periodic)
        want = p.hot_areas(wd, thr, periodic)
        ref = D.hot_area_count(w, thr, periodic=periodic)
        print(f"static hot areas n={n}: {got} (context {want}, oracle {ref})", flush=True)
        assert got == want == ref and got > 10
    h = L.lib()
    out = ctypes.c_int64()
    wd = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
    assert h.ssfm_hot_areas_static(ctypes.c_void_p(wd.data_ptr()), 4096, 1.0, 1, None,
                                   ctypes.byref(out)) == L.EINVAL
    assert b"2048" in h.ssfm_last_error()
    assert h.ssfm_hot_areas_static(None, 16, 1.0, 1, None, ctypes.byref(out)) == L.EINVAL
    p.close()
