"""The C-ABI library: loads, exports every declared symbol, host-side checks.

No test here launches a kernel; all run without a GPU.
"""
import ctypes
import os
import re

import pytest

import workloads as W
from paper_2306_15678_amd import _lib as L
from paper_2306_15678_amd.march import desc_of

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ssfm.h")).read()
    return sorted(set(re.findall(r"\b(ssfm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    h = L.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(h, n), n
    assert set(names) == set(L._SIGS)


def test_version_and_status_strings():
    h = L.lib()
    assert h.ssfm_version() == 10000
    for s in (L.OK, L.EINVAL, L.EUNSUPPORTED, L.EHIP, L.ESTATE, L.ENONFINITE, L.EWORKSPACE):
        assert h.ssfm_strerror(s)
    assert h.ssfm_strerror(-99) == b"unknown status"


def _ws(insts, precision=32, max_steps=0, ckpt=1, kept=0):
    arr = (L.InstanceDesc * len(insts))(*[desc_of(i) for i in insts])
    out = ctypes.c_size_t()
    st = L.lib().ssfm_workspace_bytes(arr, len(insts), precision, max_steps, ckpt, kept,
                                      ctypes.byref(out))
    return st, out.value


def test_workspace_bytes_scale_with_grid_and_precision():
    c1 = W.config1()[0]
    st, b32 = _ws([c1], 32)
    assert st == 0
    st, b64 = _ws([c1], 64)
    assert st == 0 and b64 > b32 >= 3 * 128 * 128 * 8
    c2 = W.config2()[0]
    st, big = _ws([c2], 32)
    assert st == 0 and big > 3 * 1024 * 1024 * 8
    # checkpoints: store-all needs more than every-50
    st, a = _ws([c2], 32, 2000, 50)
    st2, b = _ws([c2], 32, 2000, 2000)
    assert st == 0 and st2 == 0 and b > a


def test_workspace_bytes_rejects_bad_arguments():
    c1 = W.config1()[0]
    arr = (L.InstanceDesc * 1)(desc_of(c1))
    d = arr[0]
    d.n = 100
    out = ctypes.c_size_t()
    h = L.lib()
    assert h.ssfm_workspace_bytes(arr, 1, 32, 0, 1, 0, ctypes.byref(out)) == L.EUNSUPPORTED
    assert b"grid size 100" in h.ssfm_last_error()
    d.n = 128
    d.dz = -1.0
    assert h.ssfm_workspace_bytes(arr, 1, 32, 0, 1, 0, ctypes.byref(out)) == L.EINVAL
    d.dz = 1e-3
    assert h.ssfm_workspace_bytes(arr, 1, 48, 0, 1, 0, ctypes.byref(out)) == L.EINVAL
    assert h.ssfm_workspace_bytes(arr, 0, 32, 0, 1, 0, ctypes.byref(out)) == L.EINVAL
    assert h.ssfm_workspace_bytes(arr, 1, 32, 0, 0, 0, ctypes.byref(out)) == L.EINVAL
    assert h.ssfm_workspace_bytes(None, 1, 32, 0, 1, 0, ctypes.byref(out)) == L.EINVAL
    assert h.ssfm_workspace_bytes(arr, 1, 32, 10, 2, -1, ctypes.byref(out)) == L.EINVAL


def test_screens_closer_than_a_step_are_refused():
    """Turbulence screens spaced below dz could share a step (or land before
    the first one): refused, as the oracle refuses them; at screen_dz = dz
    every screen has a step of its own."""
    c3 = W.config3(1)[0]
    arr = (L.InstanceDesc * 1)(desc_of(c3))
    d = arr[0]
    out = ctypes.c_size_t()
    h = L.lib()
    assert h.ssfm_workspace_bytes(arr, 1, 32, 0, 1, 0, ctypes.byref(out)) == L.OK
    d.screen_dz = 0.5 * d.dz
    assert h.ssfm_workspace_bytes(arr, 1, 32, 0, 1, 0, ctypes.byref(out)) == L.EINVAL
    assert b"screen_dz" in h.ssfm_last_error()
    d.screen_dz = d.dz
    assert h.ssfm_workspace_bytes(arr, 1, 32, 0, 1, 0, ctypes.byref(out)) == L.OK


def test_create_checks_workspace_before_touching_the_device():
    c1 = W.config1()[0]
    arr = (L.InstanceDesc * 1)(desc_of(c1))
    ctx = ctypes.c_void_p()
    h = L.lib()
    assert h.ssfm_create(arr, 1, 32, 0, 1, 0, None, 0, None, ctypes.byref(ctx)) == L.EWORKSPACE
    assert not ctx.value
    assert h.ssfm_create(arr, 1, 32, 0, 1, 0, ctypes.c_void_p(256), 16, None,
                         ctypes.byref(ctx)) == L.EWORKSPACE
    assert h.ssfm_create(arr, 1, 32, 0, 1, 0, ctypes.c_void_p(257), 1 << 30, None,
                         ctypes.byref(ctx)) == L.EWORKSPACE


def test_null_context_is_rejected():
    h = L.lib()
    assert h.ssfm_propagate(None, 1) == L.EINVAL
    assert h.ssfm_backward(None) == L.EINVAL
    assert h.ssfm_destroy(None) == L.OK


def test_plan_variant_counts():
    r, c = ctypes.c_int32(), ctypes.c_int32()
    for n in (128, 256, 512, 768, 1024, 2048, 4096):
        assert L.lib().ssfm_plan_variants(n, 32, ctypes.byref(r), ctypes.byref(c)) == 0
        assert r.value >= 2 and c.value >= 2
    assert L.lib().ssfm_plan_variants(100, 32, ctypes.byref(r), ctypes.byref(c)) == L.EUNSUPPORTED


def test_checkpoint_interval_keeps_trajectory_when_it_fits():
    """The whole 2000-step complex64 trajectory of the 1024^2 beam (16 GiB)
    is kept when the budget allows it, else ceil(sqrt(2000)) = 45."""
    import workloads as W
    from paper_2306_15678_amd.march import checkpoint_interval, desc_of, workspace_bytes
    d = [desc_of(W.config2()[0])]
    full = workspace_bytes(d, 32, 2000, 2000)
    assert full >= 2000 * 1024 * 1024 * 8
    assert checkpoint_interval(d, 32, 2000, budget_bytes=full) == 2000
    assert checkpoint_interval(d, 32, 2000, budget_bytes=full - 1) == 45
    assert workspace_bytes(d, 32, 2000, 45) < full // 10


def test_kept_segments_cost_their_slots():
    """Each segment kept whole by the record costs M - 1 fields; with two
    or more segments left to recompute, two banks of M - 1 fields stay."""
    c2 = W.config2()[0]
    f = 1024 * 1024 * 8
    _, b0 = _ws([c2], 32, 2000, 50, 0)
    for k in (1, 7, 38):
        st, bk = _ws([c2], 32, 2000, 50, k)
        assert st == 0 and bk - b0 == k * 49 * f
    # 40 segments: keeping 39 leaves one to recompute (one bank), keeping
    # all leaves none
    _, b39 = _ws([c2], 32, 2000, 50, 39)
    _, b40 = _ws([c2], 32, 2000, 50, 40)
    _, b99 = _ws([c2], 32, 2000, 50, 99)
    assert b39 - b0 == (39 - 1) * 49 * f and b40 == b39 and b99 == b40


def _plan(insts, precision, n_steps, budget):
    arr = (L.InstanceDesc * len(insts))(*[desc_of(i) for i in insts])
    m, k, rec = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    st = L.lib().ssfm_checkpoint_plan(arr, len(insts), precision, n_steps, budget,
                                      ctypes.byref(m), ctypes.byref(k), ctypes.byref(rec))
    return st, m.value, k.value, rec.value


def _recomputed(n, m, k):
    """Steps the backward recomputes, counted segment by segment."""
    if m >= n:
        return 0
    seg = -(-n // m)
    kept = min(k, seg)
    return sum(min(m, n - s * m) - 1 for s in range(seg - kept))


def test_checkpoint_plan_is_the_cheapest_layout_that_fits():
    """Against brute force over every (M, K) of a 60-step record of two
    beams: the plan fits the budget, its recompute count is the segment by
    segment count, and no layout that fits costs less (recomputed steps plus
    one per segment)."""
    insts = [W.config1()[0], W.config3(1)[0]]
    n = 60
    _, full = _ws(insts, 32, n, n)
    sizes = {}
    for m in range(2, n):
        seg = -(-n // m)
        for k in range(0, seg + 1):
            sizes[(m, k)] = _ws(insts, 32, n, m, k)[1]
    smallest = min(sizes.values())
    for frac in (0.15, 0.3, 0.5, 0.8):
        budget = int(smallest + frac * (full - smallest))
        st, m, k, rec = _plan(insts, 32, n, budget)
        assert st == 0, L.lib().ssfm_last_error()
        assert sizes[(m, k)] <= budget and rec == _recomputed(n, m, k)
        cost = rec + -(-n // m)
        best = min(_recomputed(n, mm, kk) + -(-n // mm)
                   for (mm, kk), b in sizes.items() if b <= budget)
        assert cost == best, (frac, m, k)
    st, m, k, rec = _plan(insts, 32, n, full)
    assert (st, m, k, rec) == (0, n, 0, 0)
    st, *_ = _plan(insts, 32, n, smallest - 1)
    assert st == L.EWORKSPACE


def test_checkpoint_plan_of_the_large_aperture_march():
    """The 4096^2, 5000-step record in 200 GiB: most of the budget holds
    whole segments, so fewer than 3/4 of the steps are recomputed (against
    all but one per segment with checkpoints alone)."""
    c5 = W.config5()[0]
    budget = 200 * 2 ** 30
    st, m, k, rec = _plan([c5], 32, c5.n_steps, budget)
    assert st == 0 and k > 0
    _, b = _ws([c5], 32, c5.n_steps, m, k)
    assert b <= budget and b > 0.95 * budget
    assert rec == _recomputed(c5.n_steps, m, k) and rec < 0.75 * c5.n_steps


def test_parameter_structs_match_the_header(tmp_path):
    """ctypes mirrors of ssfm_instance_desc and ssfm_lens have the C layout
    (sizes and field offsets from a program compiled against the header)."""
    import shutil
    import subprocess
    from paper_2306_15678_amd import _lib as L
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = {"ssfm_instance_desc": L.InstanceDesc, "ssfm_lens": L.LensParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ssfm.h"', 'int main(void) {']
    for cname, py in names.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        cname, what, val = line.split()
        py = names[cname]
        want = ctypes.sizeof(py) if what == "size" else getattr(py, what).offset
        assert int(val) == want, line
