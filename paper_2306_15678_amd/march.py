"""Python front end of the HIP split-step march (libssfm).

``Propagator`` owns one library context: a caller-owned device workspace (a
torch uint8 tensor), the torch stream the kernels run on, and the beams.
Fields cross this boundary as complex128 in SI units (sqrt(W/m^2)), either
numpy arrays (host) or CUDA tensors (device).  All arithmetic happens in
the library's kernels; torch is used only to hold memory and pick streams.
"""
from __future__ import annotations

import ctypes
import math
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


def make_desc(n: int, length: float, dz: float, *, wavelength: float, n2: float,
              terms: int, mpa_order: int = 8, beta_k: float = 0.0,
              i_ref: float = 5e17, cn2: float = 0.0, screen_dz: float = 0.0,
              n_screens: int = 0, seed: int = 0) -> L.InstanceDesc:
    d = L.InstanceDesc()
    d.n, d.mpa_order, d.terms, d.n_screens = n, mpa_order, terms, n_screens
    d.length, d.dz, d.wavelength, d.n2 = length, dz, wavelength, n2
    d.beta_k, d.i_ref, d.cn2, d.screen_dz, d.seed = beta_k, i_ref, cn2, screen_dz, seed
    return d


def desc_of(inst) -> L.InstanceDesc:
    """Descriptor from any object with the beam/grid/medium attributes
    (n, length, dz, medium.{wavelength, n2, mpa_order, beta_k, i_ref, terms},
    cn2, screen_dz, n_screens, seed)."""
    m = inst.medium
    return make_desc(inst.n, inst.length, inst.dz, wavelength=m.wavelength, n2=m.n2,
                     terms=m.terms, mpa_order=m.mpa_order, beta_k=m.beta_k,
                     i_ref=m.i_ref, cn2=getattr(inst, "cn2", 0.0),
                     screen_dz=getattr(inst, "screen_dz", 0.0),
                     n_screens=getattr(inst, "n_screens", 0),
                     seed=getattr(inst, "seed", 0))


def _ptr_where(x, dtype_np, dtype_t):
    """(pointer, where, keepalive) for a host numpy or CUDA torch buffer."""
    if isinstance(x, torch.Tensor):
        if not x.is_cuda:
            x = x.detach().numpy()
        else:
            t = x.detach()
            if t.dtype != dtype_t:
                raise TypeError(f"expected {dtype_t}, got {t.dtype}")
            t = t.contiguous()
            return ctypes.c_void_p(t.data_ptr()), L.DEVICE, t
    a = np.ascontiguousarray(x, dtype=dtype_np)
    return a.ctypes.data_as(ctypes.c_void_p), L.HOST, a


class Propagator:
    """A batch of beams marching in lock-step on one GPU."""

    def __init__(self, descs: Sequence[L.InstanceDesc], precision: int = 32,
                 max_steps: int = 0, ckpt_every: int = 1,
                 device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None, stored_segments: int = 0):
        L.lib()
        if not torch.cuda.is_available():
            raise RuntimeError("Propagator needs a GPU (HIP device); none is visible")
        self.device = torch.device(device or "cuda")
        self.descs = list(descs)
        self.n_inst = len(self.descs)
        arr = (L.InstanceDesc * self.n_inst)(*self.descs)
        self._arr = arr
        self.precision = precision
        self.max_steps = int(max_steps)
        nbytes = ctypes.c_size_t()
        L.call("ssfm_workspace_bytes", arr, self.n_inst, precision, max_steps,
               ckpt_every, stored_segments, ctypes.byref(nbytes))
        self.ws_bytes = nbytes.value
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8,
                                     device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream or torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        L.call("ssfm_create", arr, self.n_inst, precision, max_steps, ckpt_every,
               stored_segments, ctypes.c_void_p(self._ws_ptr), self.ws_bytes,
               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        self.ctx = ctx

    # ------------------------------------------------------------ lifecycle
    def close(self) -> None:
        """Destroy the context and release its workspace (also while other
        references to this object remain)."""
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            L.lib().ssfm_destroy(self.ctx)
            self.ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _n(self, i: int) -> int:
        return self.descs[i].n

    # -------------------------------------------------------------- inputs
    def set_field(self, i: int, u) -> None:
        p, w, keep = _ptr_where(u, np.complex128, torch.complex128)
        L.call("ssfm_set_field", self.ctx, i, p, w)
        if w == L.DEVICE:
            self.stream.synchronize()
        del keep

    def set_theta(self, i: int, theta: Iterable[float]) -> None:
        th = (ctypes.c_double * 8)(*[float(v) for v in theta])
        L.call("ssfm_set_theta", self.ctx, i, th)

    def gen_screens(self) -> None:
        L.call("ssfm_gen_screens", self.ctx)

    # ---------------------------------------------------------------- march
    def propagate(self, n_steps: int) -> None:
        L.call("ssfm_propagate", self.ctx, int(n_steps))

    def forward_record(self, n_steps: int) -> None:
        L.call("ssfm_forward_record", self.ctx, int(n_steps))

    def set_cotangent(self, i: int, g) -> None:
        p, w, keep = _ptr_where(g, np.complex128, torch.complex128)
        L.call("ssfm_set_cotangent", self.ctx, i, p, w)
        if w == L.DEVICE:
            self.stream.synchronize()
        del keep

    def fluence_mismatch(self, i: int, target) -> float:
        """The fluence loss of instance i's current field, after any march,
        without seeding the adjoint."""
        p, w, keep = _ptr_where(target, np.float64, torch.float64)
        out = ctypes.c_double()
        L.call("ssfm_fluence_mismatch", self.ctx, i, p, w, ctypes.byref(out))
        del keep
        return out.value

    def fluence_loss(self, i: int, target) -> float:
        p, w, keep = _ptr_where(target, np.float64, torch.float64)
        out = ctypes.c_double()
        L.call("ssfm_fluence_loss", self.ctx, i, p, w, ctypes.byref(out))
        del keep
        return out.value

    def backward(self) -> None:
        L.call("ssfm_backward", self.ctx)

    def synchronize(self) -> None:
        L.call("ssfm_synchronize", self.ctx)

    # -------------------------------------------------------------- outputs
    def _out(self, name: str, i: int, shape: Tuple[int, ...], dtype_t, device: bool,
             extra: Tuple = ()):
        n = self._n(i)
        if device:
            t = torch.empty((n, n), dtype=dtype_t, device=self.device)
            L.call(name, self.ctx, i, *extra, ctypes.c_void_p(t.data_ptr()), L.DEVICE)
            return t
        dt = np.complex128 if dtype_t == torch.complex128 else np.float64
        a = np.empty((n, n), dtype=dt)
        L.call(name, self.ctx, i, *extra, a.ctypes.data_as(ctypes.c_void_p), L.HOST)
        return a

    def field(self, i: int = 0, device: bool = False):
        return self._out("ssfm_get_field", i, (), torch.complex128, device)

    def intensity(self, i: int = 0, device: bool = False):
        return self._out("ssfm_get_intensity", i, (), torch.float64, device)

    def grad_field(self, i: int = 0, device: bool = False):
        return self._out("ssfm_get_grad_field", i, (), torch.complex128, device)

    def screen(self, i: int, s: int, device: bool = False):
        return self._out("ssfm_get_screen", i, (), torch.float64, device, extra=(s,))

    def grad_theta(self, i: int = 0) -> np.ndarray:
        g = (ctypes.c_double * 8)()
        L.call("ssfm_get_grad_theta", self.ctx, i, g)
        return np.array(list(g))

    def diag(self, i: int, n: int) -> Tuple[np.ndarray, np.ndarray]:
        pw = np.empty(n)
        pk = np.empty(n)
        L.call("ssfm_get_diag", self.ctx, i, pw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
               pk.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
        return pw, pk

    # ------------------------------------------------------------- tuning
    def set_precise_math(self, enable: bool) -> None:
        L.call("ssfm_set_precise_math", self.ctx, 1 if enable else 0)

    def set_recompute_overlap(self, enable: bool) -> None:
        """Recompute checkpointed segments on a second stream beside the
        adjoint (True) or after it on the context's stream (False, default);
        the gradients are the same bitwise."""
        L.call("ssfm_set_recompute_overlap", self.ctx, 1 if enable else 0)

    def use_graphs(self, enable: bool) -> None:
        L.call("ssfm_use_graphs", self.ctx, 1 if enable else 0)

    def select_plan(self, n: int, row_variant: int, col_variant: int) -> None:
        L.call("ssfm_select_plan", self.ctx, n, row_variant, col_variant)

    def select_adjoint_plan(self, n: int, row_variant: int, col_variant: int) -> None:
        """Variants of the adjoint passes for grid size n (-1: follow the
        forward ones)."""
        L.call("ssfm_select_adjoint_plan", self.ctx, n, row_variant, col_variant)

    def time_adjoint_passes(self, reps: int = 20):
        """(ms_col, ms_row) per launch of the adjoint column and row pass."""
        c, r = ctypes.c_double(), ctypes.c_double()
        L.call("ssfm_time_adjoint_passes", self.ctx, reps, ctypes.byref(c), ctypes.byref(r))
        return c.value, r.value

    def time_passes(self, reps: int = 20):
        """(ms_row, ms_col, bytes_row, bytes_col) per launch of one pass."""
        vals = [ctypes.c_double() for _ in range(4)]
        L.call("ssfm_time_passes", self.ctx, reps, *[ctypes.byref(v) for v in vals])
        return tuple(v.value for v in vals)

    def set_splitting(self, strang: bool) -> None:
        """Lie (default) or Strang splitting of each step; zeroes the fields."""
        L.call("ssfm_set_splitting", self.ctx, L.STRANG if strang else L.LIE)

    def set_finite_difference(self, iterations: Optional[int] = None) -> None:
        """March with the finite-difference reference scheme (Crank-Nicolson,
        `iterations` fixed-point iterations per step); zeroes the fields."""
        L.call("ssfm_set_splitting", self.ctx, L.FD)
        if iterations is not None:
            L.call("ssfm_set_fd_iterations", self.ctx, int(iterations))

    def set_screen_spectrum(self, i: int, step: Optional[Tuple[float, float]] = None) -> None:
        """Screen spectrum of instance i for the next gen_screens: Kolmogorov
        (None) or the Eq. (10) low-pass step (tau [rad^2 per mode],
        kappa_h [rad/m])."""
        if step is None:
            L.call("ssfm_set_screen_spectrum", self.ctx, i, L.SPECTRUM_KOLMOGOROV, 0.0, 0.0)
        else:
            L.call("ssfm_set_screen_spectrum", self.ctx, i, L.SPECTRUM_STEP,
                   float(step[0]), float(step[1]))

    def set_subharmonics(self, i: int, levels: int) -> None:
        """Subharmonic levels (0-8) added to instance i's screens by the next
        gen_screens: the power below the window's fundamental 1/L."""
        L.call("ssfm_set_subharmonics", self.ctx, i, int(levels))

    def apply_lens(self, i: int, lens: L.LensParams) -> None:
        """Apply the effective-lens screen to instance i's current field."""
        L.call("ssfm_apply_lens", self.ctx, i, ctypes.byref(lens))

    def lens_vjp(self, i: int, lens: L.LensParams, u_in, g_out):
        """(g_in, grad) of the lens applied to u_in, for the output cotangent
        g_out (G = dL/dRe U + i dL/dIm U): g_in on the device, grad =
        dL/d(c1, c2, then amplitude, frequency, phase of each real segment,
        then of each imaginary one)."""
        n = self._n(i)
        u = torch.as_tensor(u_in).to(self.device, torch.complex128).contiguous()
        g = torch.as_tensor(g_out).to(self.device, torch.complex128).contiguous()
        if u.shape != (n, n) or g.shape != (n, n):
            raise ValueError(f"u_in and g_out must be {n} x {n}")
        g_in = torch.empty_like(u)
        k = 2 + 3 * (lens.n_re + lens.n_im)
        grad = (ctypes.c_double * k)()
        torch.cuda.synchronize(self.device)     # inputs written on torch's streams
        L.call("ssfm_lens_vjp", self.ctx, i, ctypes.byref(lens), ctypes.c_void_p(u.data_ptr()),
               ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(g_in.data_ptr()), grad, k)
        return g_in, np.array(list(grad))

    def hot_areas(self, w: torch.Tensor, threshold: float, periodic: bool = True) -> int:
        """Number of hot areas: 4-connected regions with w >= threshold
        [W/m^2] of an n x n float64 fluence on this device."""
        w = w.to(device=self.device, dtype=torch.float64).contiguous()
        out = ctypes.c_int64()
        L.call("ssfm_hot_areas", self.ctx, ctypes.c_void_p(w.data_ptr()), w.shape[0],
               float(threshold), 1 if periodic else 0, ctypes.byref(out))
        return out.value

    def measure_vector(self, w: torch.Tensor, length: float, w_p: float,
                       periodic: bool = True) -> np.ndarray:
        """P = (Q(1,0), Q(1,1), Q(2,0), Q(2,1), max w, N_ha(w >= w_p)) of an
        n x n float64 fluence on this device (the GA's measure vector)."""
        w = w.to(device=self.device, dtype=torch.float64).contiguous()
        out = (ctypes.c_double * L.MEASURE_LEN)()
        L.call("ssfm_measure_vector", self.ctx, ctypes.c_void_p(w.data_ptr()), w.shape[0],
               float(length), float(w_p), 1 if periodic else 0, out)
        return np.array(list(out))

    def measure_distance(self, i: int, p0: Sequence[float], w_p: float,
                         periodic: bool = True) -> Tuple[float, np.ndarray]:
        """(d, P): the relative Euclidean distance of instance i's current
        fluence's measure vector P from p0, and P."""
        ref = (ctypes.c_double * L.MEASURE_LEN)(*[float(v) for v in p0])
        d = ctypes.c_double()
        out = (ctypes.c_double * L.MEASURE_LEN)()
        L.call("ssfm_measure_distance", self.ctx, i, float(w_p), 1 if periodic else 0, ref,
               ctypes.byref(d), out)
        return d.value, np.array(list(out))

    def moment(self, w: torch.Tensor, length: float, p: float, m: int) -> float:
        """Q(p, m) = sum w^p (x^2 + y^2)^m dx^2 of an n x n float64 fluence."""
        w = w.to(device=self.device, dtype=torch.float64).contiguous()
        out = ctypes.c_double()
        L.call("ssfm_moment", self.ctx, ctypes.c_void_p(w.data_ptr()), w.shape[0],
               float(length), float(p), int(m), ctypes.byref(out))
        return out.value

    def set_pass_timing(self, every: int) -> None:
        """Sample the row/column pass durations every ``every`` steps of each
        forward march (0: off)."""
        L.call("ssfm_set_pass_timing", self.ctx, int(every))

    def pass_times(self):
        """(ms_row, ms_col, n_samples) of the most recent forward march."""
        r, c, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        L.call("ssfm_pass_times", self.ctx, ctypes.byref(r), ctypes.byref(c), ctypes.byref(n))
        return r.value, c.value, n.value

    def adjoint_pass_times(self):
        """(ms_col, ms_row, n_samples) of the adjoint passes sampled in the
        most recent backward (pass timing on)."""
        c, r, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        L.call("ssfm_adjoint_pass_times", self.ctx, ctypes.byref(c), ctypes.byref(r),
               ctypes.byref(n))
        return c.value, r.value, n.value

    def block_mean(self, src: torch.Tensor, b: int) -> torch.Tensor:
        n = src.shape[0]
        src = src.contiguous()
        out = torch.empty((n // b, n // b), dtype=torch.float64, device=self.device)
        L.call("ssfm_block_mean", self.ctx, ctypes.c_void_p(src.data_ptr()), n, b,
               ctypes.c_void_p(out.data_ptr()))
        return out


def hot_areas_static(w: torch.Tensor, threshold: float, periodic: bool = True,
                     stream: Optional[torch.cuda.Stream] = None) -> int:
    """Hot-area count of an n x n float64 fluence on the current device
    without a context or any device allocation (the library's fixed
    scratch; n <= 2048), on ``stream`` (default: torch's current one)."""
    w = w.to(dtype=torch.float64).contiguous()
    st = stream or torch.cuda.current_stream(w.device)
    out = ctypes.c_int64()
    L.call("ssfm_hot_areas_static", ctypes.c_void_p(w.data_ptr()), w.shape[0],
           float(threshold), 1 if periodic else 0, ctypes.c_void_p(st.cuda_stream),
           ctypes.byref(out))
    return out.value


def make_lens(l_dif: float, w_l: float, c1: float, c2: float,
              re: Sequence[Sequence[float]] = (), im: Sequence[Sequence[float]] = ()
              ) -> L.LensParams:
    """Effective-lens parameters: filter l_dif [m^2], trimming level w_l
    [W/m^2], cubic lens field w = c1 (r^3 - c2), and up to 8 segments
    (r_end [m], amplitude, frequency [1/m], phase) of the real and the
    imaginary profile."""
    if len(re) > 8 or len(im) > 8:
        raise ValueError("at most 8 segments per part")
    p = L.LensParams()
    p.l_dif, p.w_l, p.c1, p.c2 = float(l_dif), float(w_l), float(c1), float(c2)
    p.n_re, p.n_im = len(re), len(im)
    for j, row in enumerate(re):
        for k in range(4):
            p.re[j][k] = float(row[k])
    for j, row in enumerate(im):
        for k in range(4):
            p.im[j][k] = float(row[k])
    return p


def march_with_lens(prop: "Propagator", i: int, n_steps: int, w_pf: float,
                    lens: L.LensParams, chunk: int = 10) -> Optional[int]:
    """March n_steps in chunks; after the first chunk in which the peak
    intensity of instance i reaches the pre-filamentation level w_pf
    [W/m^2], apply the effective lens to instance i once.  Returns the step
    count at which it was applied, or None."""
    done, applied = 0, None
    while done < n_steps:
        k = min(chunk, n_steps - done)
        prop.propagate(k)
        done += k
        if applied is None:
            _, peak = prop.diag(i, k)
            if float(np.max(peak)) >= w_pf:
                prop.apply_lens(i, lens)
                applied = done
    return applied


def hot_area_trace(prop: "Propagator", i: int, n_steps: int, every: int,
                   threshold: float, periodic: bool = True) -> List[int]:
    """N_ha along the optical path: march instance i's context n_steps steps
    from its current state, counting hot areas (w >= threshold) every
    `every` steps (all instances of the context advance together)."""
    counts = []
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        prop.propagate(k)
        done += k
        counts.append(prop.hot_areas(prop.intensity(i, device=True), threshold, periodic))
    return counts


def workspace_bytes(descs: Sequence[L.InstanceDesc], precision: int, max_steps: int,
                    ckpt_every: int, stored_segments: int = 0) -> int:
    """Device workspace a context with these arguments needs."""
    arr = (L.InstanceDesc * len(descs))(*descs)
    nbytes = ctypes.c_size_t()
    L.call("ssfm_workspace_bytes", arr, len(descs), precision, max_steps, ckpt_every,
           stored_segments, ctypes.byref(nbytes))
    return nbytes.value


def checkpoint_plan(descs: Sequence[L.InstanceDesc], precision: int, n_steps: int,
                    budget_bytes: Optional[int] = None) -> Tuple[int, int, int]:
    """(M, K, recomputed steps) for a recorded march of n_steps whose
    workspace fits the budget (default: three quarters of the free device
    memory): every pre-screen field kept when that fits, else checkpoints
    every M steps with the last K segments kept whole, chosen to recompute
    the fewest steps (ssfm_checkpoint_plan)."""
    if budget_bytes is None:
        budget_bytes = torch.cuda.mem_get_info()[0] * 3 // 4
    arr = (L.InstanceDesc * len(descs))(*descs)
    m, k, rec = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    L.call("ssfm_checkpoint_plan", arr, len(descs), precision, n_steps, int(budget_bytes),
           ctypes.byref(m), ctypes.byref(k), ctypes.byref(rec))
    return m.value, k.value, rec.value


def checkpoint_interval(descs: Sequence[L.InstanceDesc], precision: int, n_steps: int,
                        budget_bytes: Optional[int] = None) -> int:
    """Checkpoint interval M for a recorded march of n_steps: n_steps (every
    pre-screen field kept, no recompute in the backward) when that workspace
    fits the budget (default: half the free device memory), else
    ceil(sqrt(n_steps)) (checkpoints plus two banks of one segment)."""
    if budget_bytes is None:
        budget_bytes = torch.cuda.mem_get_info()[0] // 2
    if workspace_bytes(descs, precision, n_steps, n_steps) <= budget_bytes:
        return n_steps
    return max(1, math.isqrt(n_steps - 1) + 1)


def plan_variants(n: int, precision: int = 32) -> Tuple[int, int]:
    """(row variants, column variants) compiled for grid size n."""
    r, c = ctypes.c_int32(), ctypes.c_int32()
    L.call("ssfm_plan_variants", n, precision, ctypes.byref(r), ctypes.byref(c))
    return r.value, c.value
