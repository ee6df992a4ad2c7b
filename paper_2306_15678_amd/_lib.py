"""ctypes binding of libssfm.so (the C ABI declared in include/ssfm.h).

Argument marshalling only: every step of the march runs in the library's
HIP kernels.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t,
                    c_uint32, c_uint64, c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssfm.so")

OK, EINVAL, EUNSUPPORTED, EHIP, ESTATE, ENONFINITE, EWORKSPACE = 0, -1, -2, -3, -4, -5, -6
KERR, MPA, PLASMA, ANSATZ, TURB = 1, 2, 4, 8, 16
FP32, FP64 = 32, 64
HOST, DEVICE = 0, 1


class InstanceDesc(ctypes.Structure):
    """Mirror of ssfm_instance_desc."""

    _fields_ = [
        ("n", c_int32), ("mpa_order", c_int32), ("terms", c_uint32),
        ("n_screens", c_int32), ("length", c_double), ("dz", c_double),
        ("wavelength", c_double), ("n2", c_double), ("beta_k", c_double),
        ("i_ref", c_double), ("cn2", c_double), ("screen_dz", c_double),
        ("seed", c_uint64),
    ]


class SsfmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status} ({detail})")
        self.status = status


SPECTRUM_KOLMOGOROV, SPECTRUM_STEP = 0, 1
MEASURE_LEN = 6
LIE, STRANG, FD = 0, 1, 2


class LensParams(ctypes.Structure):
    """Mirror of ssfm_lens (effective-lens screen parameters, SI)."""
    _fields_ = [("l_dif", c_double), ("w_l", c_double), ("c1", c_double), ("c2", c_double),
                ("n_re", c_int32), ("n_im", c_int32),
                ("re", (c_double * 4) * 8), ("im", (c_double * 4) * 8)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "ssfm_version": (c_int32, []),
    "ssfm_strerror": (c_char_p, [c_int32]),
    "ssfm_last_error": (c_char_p, []),
    "ssfm_workspace_bytes": (c_int32, [POINTER(InstanceDesc), c_int32, c_int32, c_int64,
                                       c_int32, c_int32, POINTER(c_size_t)]),
    "ssfm_checkpoint_plan": (c_int32, [POINTER(InstanceDesc), c_int32, c_int32, c_int64,
                                       c_size_t, POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_int64)]),
    "ssfm_create": (c_int32, [POINTER(InstanceDesc), c_int32, c_int32, c_int64, c_int32,
                              c_int32, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "ssfm_destroy": (c_int32, [c_void_p]),
    "ssfm_set_field": (c_int32, [c_void_p, c_int32, c_void_p, c_int32]),
    "ssfm_set_theta": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "ssfm_gen_screens": (c_int32, [c_void_p]),
    "ssfm_get_screen": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int32]),
    "ssfm_propagate": (c_int32, [c_void_p, c_int64]),
    "ssfm_get_field": (c_int32, [c_void_p, c_int32, c_void_p, c_int32]),
    "ssfm_get_intensity": (c_int32, [c_void_p, c_int32, c_void_p, c_int32]),
    "ssfm_get_diag": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                c_int64]),
    "ssfm_forward_record": (c_int32, [c_void_p, c_int64]),
    "ssfm_set_cotangent": (c_int32, [c_void_p, c_int32, c_void_p, c_int32]),
    "ssfm_fluence_loss": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, POINTER(c_double)]),
    "ssfm_backward": (c_int32, [c_void_p]),
    "ssfm_get_grad_field": (c_int32, [c_void_p, c_int32, c_void_p, c_int32]),
    "ssfm_get_grad_theta": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "ssfm_block_mean": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p]),
    "ssfm_use_graphs": (c_int32, [c_void_p, c_int32]),
    "ssfm_set_precise_math": (c_int32, [c_void_p, c_int32]),
    "ssfm_set_recompute_overlap": (c_int32, [c_void_p, c_int32]),
    "ssfm_plan_variants": (c_int32, [c_int32, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "ssfm_select_plan": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "ssfm_time_passes": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                   POINTER(c_double), POINTER(c_double)]),
    "ssfm_apply_lens": (c_int32, [c_void_p, c_int32, POINTER(LensParams)]),
    "ssfm_lens_vjp": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_int32]),
    "ssfm_set_screen_spectrum": (c_int32, [c_void_p, c_int32, c_int32, c_double, c_double]),
    "ssfm_set_subharmonics": (c_int32, [c_void_p, c_int32, c_int32]),
    "ssfm_set_fd_iterations": (c_int32, [c_void_p, c_int32]),
    "ssfm_set_splitting": (c_int32, [c_void_p, c_int32]),
    "ssfm_fluence_mismatch": (c_int32, [c_void_p, c_int32, c_void_p, c_int32,
                                        POINTER(c_double)]),
    "ssfm_hot_areas": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_int32,
                                 POINTER(c_int64)]),
    "ssfm_hot_areas_static": (c_int32, [c_void_p, c_int32, c_double, c_int32, c_void_p,
                                        POINTER(c_int64)]),
    "ssfm_measure_vector": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_double, c_int32,
                                      POINTER(c_double)]),
    "ssfm_measure_distance": (c_int32, [c_void_p, c_int32, c_double, c_int32, POINTER(c_double),
                                        POINTER(c_double), POINTER(c_double)]),
    "ssfm_moment": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_double, c_int32,
                              POINTER(c_double)]),
    "ssfm_set_pass_timing": (c_int32, [c_void_p, c_int32]),
    "ssfm_pass_times": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double),
                                  POINTER(c_int32)]),
    "ssfm_adjoint_pass_times": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double),
                                          POINTER(c_int32)]),
    "ssfm_select_adjoint_plan": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "ssfm_time_adjoint_passes": (c_int32, [c_void_p, c_int32, POINTER(c_double),
                                           POINTER(c_double)]),
    "ssfm_synchronize": (c_int32, [c_void_p]),
}


def lib() -> ctypes.CDLL:
    """The loaded library; raises if libssfm.so is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2306_15678_amd.build` "
                "(there is no fallback implementation)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int, where: str) -> None:
    if status != OK:
        h = lib()
        detail = (h.ssfm_last_error() or b"").decode() or h.ssfm_strerror(status).decode()
        raise SsfmError(status, where, detail)


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args), name)
