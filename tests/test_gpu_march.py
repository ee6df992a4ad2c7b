"""GPU parity of the HIP split-step march against the FP64 oracle.

Every test runs the library through its C ABI (via the ctypes binding) on
seeded synthetic inputs from ``workloads`` and compares with ``oracle`` on
the same inputs.  Tolerances: complex128 kernels agree with the oracle to
rounding (rel L2 <= 1e-11 after the stated steps); complex64 kernels to
the FP32 rounding floor of the same march (stated per test).
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W
from oracle import march as M
from oracle import turbulence as T

pytestmark = pytest.mark.gpu


def _prop(insts, precision, **kw):
    from paper_2306_15678_amd.march import Propagator, desc_of
    return Propagator([desc_of(i) for i in insts], precision=precision, **kw)


def _maxrel(a, b):
    """Largest pointwise error over the largest reference magnitude: where a
    localised error shows that a global relative L2 norm would dilute."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# Bound of _maxrel beside a relative-L2 tolerance.  Rounding spreads over
# the beam, so the pointwise maximum sits 2.5-10x above the relative L2
# (measured: 2.6-10 in FP32, 5.7 in FP64 on the 1024^2 batch beam); an error
# confined to a few points instead leaves the L2 norm near its floor while
# its pointwise maximum exceeds this bound.
MAX_OVER_L2 = 10.0


def _report(name, **vals):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                         for k, v in vals.items()), flush=True)


# ------------------------------------------------------------------ C1
# Rounding floors of this march, from tests/golden/floor_c1.json (written by
# tests/golden/calibrate_floor.py c1, which runs the oracle and an
# independent complex64 peer of the same map on the CPU).  The beam
# collapses near step 110 (Kerr only, no arrest); after that the march is
# chaotic and every floor grows ~1000x.
#                            step 100 field / fluence    step 200 field / fluence
#   FP64 per-step rounding   1.8e-14 / 2.6e-14             2.7e-11 / 5.0e-12
#   FP32 per-step rounding   7.0e-6  / 1.0e-5              1.2e-2  / 2.2e-3
#   FP32 peer vs oracle      5.0e-5  / 7.3e-5              4.4e-2  / 8.2e-3
# Tolerance: FP64 10x its floor; FP32 5x the larger FP32 floor (the peer).
C1_TOL = {64: {100: (2e-13, 3e-13), 200: (3e-10, 5e-11)},
          32: {100: (2.5e-4, 3.7e-4), 200: (2.2e-1, 4.1e-2)}}


@pytest.mark.parametrize("precision", [64, 32])
def test_config1_full_march(precision):
    """128^2 Kerr-only, 200 steps (the CPU-scale workload): field, fluence,
    power and peak against the oracle before and after the collapse."""
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    p = _prop([inst], precision)
    p.set_field(0, u0)
    u = u0
    pw_all, pk_all = [], []
    for stop in (100, 200):
        ref = M.march(u, inst, n_steps=100)
        u = ref.field
        p.propagate(100)
        got = p.field(0)
        pw, pk = p.diag(0, 100)
        pw_all += list(pw / ref.power - 1)
        pk_all += list(pk / ref.peak - 1)
        err = M.rel_l2(got, ref.field)
        ferr = M.rel_l2(np.abs(got) ** 2, np.abs(ref.field) ** 2)
        emax = _maxrel(got, ref.field)
        _report(f"c1 fp{precision} step {stop}", field=err, fluence=ferr, field_max=emax)
        tf, tw = C1_TOL[precision][stop]
        assert err < tf and ferr < tw and emax < MAX_OVER_L2 * tf
    perr = float(np.max(np.abs(pw_all)))
    _report(f"c1 fp{precision}", power=perr, peak=float(np.max(np.abs(pk_all))))
    assert perr < (1e-12 if precision == 64 else 1e-4)


# -------------------------------------------------- every size, all terms
def _strong(n, terms, theta=None, n_steps=6, length=4e-3, power=400 * W.P_CR, **kw):
    return W.Instance(n=n, length=length, dz=0.01, n_steps=n_steps,
                      medium=W.Medium(terms=terms), w0=0.5e-3, power=power,
                      sigma=0.2, seed=100 + n, theta=theta, **kw)


SIZES = [128, 256, 512, 768, 1024, 2048]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("precision", [64, 32])
def test_every_size_all_screen_terms(n, precision):
    terms = W.KPM | W.TERM_ANSATZ
    theta = tuple(np.array(W.THETA0) + W.random_theta(n, 0.2))
    inst = _strong(n, terms, theta=theta)
    u0 = W.initial_field(inst)
    ref = M.march(u0, inst)
    p = _prop([inst], precision)
    p.set_field(0, u0)
    p.set_theta(0, theta)
    p.propagate(inst.n_steps)
    got = p.field(0)
    err = M.rel_l2(got, ref.field)
    emax = _maxrel(got, ref.field)
    pw, pk = p.diag(0, inst.n_steps)
    perr = float(np.max(np.abs(pw / ref.power - 1)))
    _report(f"n={n} fp{precision}", field=err, field_max=emax, power=perr,
            peak_x=float(ref.peak.max() / W.I_A))
    tol = 1e-11 if precision == 64 else 2e-5
    assert err < tol
    assert emax < MAX_OVER_L2 * tol
    assert perr < (1e-12 if precision == 64 else 2e-6)


# ------------------------------------------------------------ screens
@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 2e-6)])
def test_turbulence_screens_match_oracle(precision, tol):
    inst = _strong(256, W.TERM_KERR | W.TERM_TURB, cn2=1e-12, screen_dz=0.02,
                   n_screens=5)
    want = T.instance_screens(inst)
    p = _prop([inst], precision)
    p.gen_screens()
    steps = inst.screen_steps()
    for s in range(inst.n_screens):
        got = p.screen(0, s)
        ref = want[steps[s]]
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        _report(f"screen {s} fp{precision}", maxrel=err, rms=float(np.std(ref)))
        assert err < tol


@pytest.mark.parametrize("precision,tol", [(64, 1e-11), (32, 2e-5)])
def test_march_with_turbulence_matches_oracle(precision, tol):
    inst = _strong(512, W.KPM | W.TERM_TURB, n_steps=9, cn2=3e-13,
                   screen_dz=0.03, n_screens=3)  # z_s/dz = 1.5, 4.5, 7.5: ties round up
    u0 = W.initial_field(inst)
    screens = T.instance_screens(inst)
    ref = M.march(u0, inst, screens=screens)
    p = _prop([inst], precision)
    p.gen_screens()
    p.set_field(0, u0)
    p.propagate(inst.n_steps)
    err = M.rel_l2(p.field(0), ref.field)
    _report(f"turb march fp{precision}", field=err)
    assert err < tol


# ------------------------------------------------------ batch, determinism
def test_batch_of_uneven_beams_equals_each_alone():
    a = _strong(256, W.KPM, n_steps=5)
    b = _strong(512, W.KPM, n_steps=5, power=150 * W.P_CR)
    c = dataclasses.replace(_strong(256, W.KPM, n_steps=5), seed=999)
    insts = [a, b, c]
    fields = [W.initial_field(i) for i in insts]
    batch = _prop(insts, 32)
    for k, u in enumerate(fields):
        batch.set_field(k, u)
    batch.propagate(5)
    for k, (inst, u) in enumerate(zip(insts, fields)):
        alone = _prop([inst], 32)
        alone.set_field(0, u)
        alone.propagate(5)
        assert np.array_equal(batch.field(k), alone.field(0)), k


def test_runs_are_bitwise_deterministic_and_graphs_match_eager():
    inst = _strong(1024, W.KPM, n_steps=12)
    u0 = W.initial_field(inst)
    outs = []
    for graphs in (True, True, False):
        p = _prop([inst], 32)
        p.use_graphs(graphs)
        p.set_field(0, u0)
        p.propagate(inst.n_steps)
        outs.append((p.field(0), p.diag(0, inst.n_steps)))
    for f, (pw, pk) in outs[1:]:
        assert np.array_equal(f, outs[0][0])
        assert np.array_equal(pw, outs[0][1][0]) and np.array_equal(pk, outs[0][1][1])


def test_propagate_in_chunks_equals_one_call():
    inst = _strong(256, W.KPM | W.TERM_TURB, n_steps=10, cn2=3e-13, screen_dz=0.03,
                   n_screens=3)
    u0 = W.initial_field(inst)
    p1 = _prop([inst], 32)
    p1.gen_screens()
    p1.set_field(0, u0)
    p1.propagate(10)
    p2 = _prop([inst], 32)
    p2.gen_screens()
    p2.set_field(0, u0)
    for k in (3, 4, 3):
        p2.propagate(k)
    assert np.array_equal(p1.field(0), p2.field(0))


# ------------------------------------------------------------- gradients
def _grad_case(n=256, turb=False):
    terms = W.KPM | W.TERM_ANSATZ
    kw = {}
    if turb:
        terms |= W.TERM_TURB
        kw = dict(cn2=3e-13, screen_dz=0.03, n_screens=3)
    theta = tuple(np.array(W.THETA0) + W.random_theta(7, 0.1))
    inst = _strong(n, terms, theta=theta, n_steps=8, power=200 * W.P_CR, **kw)
    return inst


@pytest.mark.parametrize("turb", [False, True])
@pytest.mark.parametrize("precision,ckpt", [(64, 3), (64, 100), (32, 3), (32, 100)])
def test_gradient_matches_oracle(precision, ckpt, turb):
    inst = _grad_case(turb=turb)
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    screens = T.instance_screens(inst) if turb else None
    loss, g_u0, g_th = M.gradient(u0, inst, screens=screens,
                                  cotangent=lambda u: M.fluence_loss(u, target))
    p = _prop([inst], precision, max_steps=inst.n_steps, ckpt_every=ckpt)
    if turb:
        p.gen_screens()
    p.set_field(0, u0)
    p.set_theta(0, inst.theta)
    p.forward_record(inst.n_steps)
    gl = p.fluence_loss(0, target)
    p.backward()
    gg = p.grad_field(0)
    gt = p.grad_theta(0)
    lerr = abs(gl / loss - 1)
    ferr = M.rel_l2(gg, g_u0)
    terr = float(np.max(np.abs(gt - g_th)) / np.max(np.abs(g_th)))
    _report(f"grad fp{precision} M={ckpt} turb={turb}", loss=lerr, g_u0=ferr, g_theta=terr)
    tol = 1e-10 if precision == 64 else 1e-4
    assert lerr < tol and ferr < tol and terr < tol


@pytest.mark.parametrize("graphs", [True, False])
def test_checkpointed_and_stored_adjoints_are_bitwise_equal(graphs):
    """3 segments, each recomputed after the adjoint of the next one or
    (overlap) on a second stream beside it, against all steps stored; the
    overlap setting also switched on a context whose backward sweep was
    already captured."""
    inst = _grad_case()
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    res = []
    for ckpt, overlap in ((3, False), (3, True), (100, False)):
        p = _prop([inst], 32, max_steps=inst.n_steps, ckpt_every=ckpt)
        p.use_graphs(graphs)
        for ov in ((not overlap, overlap) if ckpt == 3 else (overlap,)):
            p.set_recompute_overlap(ov)
            p.set_field(0, u0)
            p.set_theta(0, inst.theta)
            p.forward_record(inst.n_steps)
            p.fluence_loss(0, target)
            p.backward()
        res.append((p.grad_field(0), p.grad_theta(0)))
    for r in res[:2]:
        assert np.array_equal(r[0], res[2][0])
        assert np.array_equal(r[1], res[2][1])


def test_external_cotangent_matches_loss_seed():
    inst = _grad_case()
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    p = _prop([inst], 64, max_steps=inst.n_steps, ckpt_every=4)
    p.set_field(0, u0)
    p.set_theta(0, inst.theta)
    p.forward_record(inst.n_steps)
    u_n = p.field(0)
    _, g = M.fluence_loss(u_n, target)
    p.set_cotangent(0, g)
    p.backward()
    g1, t1 = p.grad_field(0), p.grad_theta(0)
    p.fluence_loss(0, target)
    p.backward()
    g2, t2 = p.grad_field(0), p.grad_theta(0)
    assert M.rel_l2(g1, g2) < 1e-12
    assert np.max(np.abs(t1 - t2)) < 1e-12 * np.max(np.abs(t2))


def test_autograd_function_matches_oracle_gradient():
    """torch.autograd through the library: a loss written in torch on U_N,
    gradients w.r.t. U0 and theta against the oracle (FP64 kernels)."""
    import torch
    from paper_2306_15678_amd.autograd import march

    inst = _grad_case(n=128)
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 9)
    loss_o, g_u0, g_th = M.gradient(u0, inst, cotangent=lambda u: M.fluence_loss(u, target))
    p = _prop([inst], 64, max_steps=inst.n_steps, ckpt_every=3)
    dev = torch.device("cuda")
    tu = torch.from_numpy(u0).to(dev).requires_grad_(True)
    tth = torch.tensor(inst.theta, dtype=torch.float64, device=dev, requires_grad=True)
    tt = torch.from_numpy(target).to(dev)
    u_n = march(tu, tth, p, inst.n_steps)
    inten = (u_n * u_n.conj()).real
    loss = ((inten - tt) ** 2).sum() / (tt ** 2).sum()
    loss.backward()
    lerr = abs(loss.item() / loss_o - 1)
    ferr = M.rel_l2(tu.grad.cpu().numpy(), g_u0)
    terr = float(np.max(np.abs(tth.grad.cpu().numpy() - g_th)) / np.max(np.abs(g_th)))
    _report("autograd fp64", loss=lerr, g_u0=ferr, g_theta=terr)
    assert lerr < 1e-10 and ferr < 1e-10 and terr < 1e-10


@pytest.mark.parametrize("n", [128, 256, 512, 768, 1024, 2048, 4096])
def test_every_tile_variant_matches_oracle(n):
    """Each compiled row and column variant (points per thread, lines per
    workgroup, radix plan, late twiddles, occupancy target) computes the same
    march: FP64 kernels against the oracle to rounding, 3 steps with every
    screen term and two turbulence screens (z_s/dz = 0.55, 1.65: after steps 0 and
    1).  A variant whose tile does not fit a workgroup in FP64 (not built for
    it) is checked in FP32 against the oracle to the FP32 tolerance of the
    all-terms march (2e-5)."""
    from paper_2306_15678_amd._lib import EUNSUPPORTED, SsfmError
    from paper_2306_15678_amd.march import plan_variants
    terms = W.KPM | W.TERM_ANSATZ | W.TERM_TURB
    theta = tuple(np.array(W.THETA0) + W.random_theta(n + 1, 0.2))
    inst = _strong(n, terms, theta=theta, n_steps=3, cn2=3e-13, screen_dz=0.011, n_screens=2)
    assert list(inst.screen_steps()) == [0, 1]
    u0 = W.initial_field(inst)
    ref = M.march(u0, inst, screens=T.instance_screens(inst))
    n_row, n_col = plan_variants(n, 64)
    combos = [(r, 0) for r in range(n_row)] + [(0, c) for c in range(1, n_col)]
    props = {}
    for precision in (64, 32):
        props[precision] = _prop([inst], precision)
        props[precision].set_theta(0, theta)
        props[precision].gen_screens()
    for r, c in combos:
        for precision, tol in ((64, 1e-11), (32, 2e-5)):
            p = props[precision]
            try:
                p.select_plan(n, r, c)
            except SsfmError as e:
                assert precision == 64 and e.status == EUNSUPPORTED
                continue
            p.set_field(0, u0)
            p.propagate(inst.n_steps)
            err = M.rel_l2(p.field(0), ref.field)
            _report(f"variant n={n} row={r} col={c} fp{precision}", field=err)
            assert err < tol, (r, c, precision)
            if precision == 64:
                break


# ------------------------------------------- adjoint row-pass variants
# Every row variant of the large grids (the persistent pipelined ones
# included: complex64 only) as the forward and the adjoint row pass of a
# recorded march with every screen term, the ansatz and two turbulence
# screens (after steps 0 and 1), 3 steps, fluence loss, backward.
def _adjoint_variant_case(n):
    terms = W.KPM | W.TERM_ANSATZ | W.TERM_TURB
    theta = tuple(np.array(W.THETA0) + W.random_theta(n + 3, 0.2))
    inst = _strong(n, terms, theta=theta, n_steps=3, cn2=3e-13, screen_dz=0.011, n_screens=2)
    assert list(inst.screen_steps()) == [0, 1]
    return inst, W.initial_field(inst), W.synthetic_target(inst, 5)


def _fwd_adj(p, inst, u0, target):
    p.set_field(0, u0)
    p.set_theta(0, inst.theta)
    p.forward_record(inst.n_steps)
    loss = p.fluence_loss(0, target)
    p.backward()
    return loss, p.grad_field(0), p.grad_theta(0)


@pytest.fixture(scope="module", params=[1024, 2048])
def adj_oracle(request):
    inst, u0, target = _adjoint_variant_case(request.param)
    screens = T.instance_screens(inst)
    return (inst, u0, target), M.gradient(u0, inst, screens=screens,
                                          cotangent=lambda u: M.fluence_loss(u, target))


def test_every_variant_adjoint_matches_oracle(adj_oracle):
    """FP32 forward + adjoint with each row variant used for both row passes
    (column variant 0), then each column variant for both column passes (row
    variant 0), against the FP64 oracle gradient: loss, gradient of U0 and
    of theta to the FP32 gradient tolerance (1e-4, as for the 256^2
    gradient case), the field gradient also pointwise."""
    from paper_2306_15678_amd.march import plan_variants
    (inst, u0, target), (loss_o, g_u0, g_th) = adj_oracle
    n = inst.n
    n_row, n_col = plan_variants(n, 32)
    p = _prop([inst], 32, max_steps=inst.n_steps, ckpt_every=2)
    p.gen_screens()
    combos = [(r, 0) for r in range(n_row)] + [(0, c) for c in range(1, n_col)]
    for r, c in combos:
        p.select_plan(n, r, c)
        p.select_adjoint_plan(n, -1, -1)
        loss, gg, gt = _fwd_adj(p, inst, u0, target)
        lerr = abs(loss / loss_o - 1)
        ferr = M.rel_l2(gg, g_u0)
        fmax = _maxrel(gg, g_u0)
        terr = float(np.max(np.abs(gt - g_th)) / np.max(np.abs(g_th)))
        _report(f"adjoint variants n={n} row={r} col={c}", loss=lerr, g_u0=ferr,
                g_u0_max=fmax, g_theta=terr)
        assert lerr < 1e-4 and ferr < 1e-4 and terr < 1e-4, (r, c)
        assert fmax < MAX_OVER_L2 * 1e-4, (r, c)


def test_precise_math_forward_adjoint_matches_oracle(adj_oracle):
    """ssfm_set_precise_math (library sine and cosine in the screens) with the
    last row and column variants of the size (the persistent pipelined ones
    at 2048^2, which hand such launches to the plain kernels): FP32 forward
    + adjoint against the FP64 oracle gradient to the FP32 gradient
    tolerance; the setting also applies to a march whose steps were already
    captured in graphs (the captured steps are dropped)."""
    from paper_2306_15678_amd.march import plan_variants
    (inst, u0, target), (loss_o, g_u0, g_th) = adj_oracle
    n = inst.n
    n_row, n_col = plan_variants(n, 32)
    p = _prop([inst], 32, max_steps=inst.n_steps, ckpt_every=2)
    p.gen_screens()
    p.select_plan(n, n_row - 1, n_col - 1)
    fast = _fwd_adj(p, inst, u0, target)
    p.set_precise_math(True)
    loss, gg, gt = _fwd_adj(p, inst, u0, target)
    lerr = abs(loss / loss_o - 1)
    ferr = M.rel_l2(gg, g_u0)
    terr = float(np.max(np.abs(gt - g_th)) / np.max(np.abs(g_th)))
    _report(f"precise math n={n} row={n_row - 1} col={n_col - 1}", loss=lerr, g_u0=ferr,
            g_theta=terr, vs_fast=M.rel_l2(gg, fast[1]))
    assert lerr < 1e-4 and ferr < 1e-4 and terr < 1e-4
    assert not np.array_equal(gg, fast[1])


def test_every_variant_adjoint_4096_agrees():
    """At 4096^2 (FP64 oracle too slow for every variant): each row variant's
    and each column variant's FP32 forward + adjoint against variants
    (0, 0), to a few FP32 roundings of the 3-step march (the radix plans
    round differently); the pipelined variants also against the plain kernel
    of the same radices and threads (same arithmetic per point; the compiler
    may fuse a multiply and an add differently in the two kernels, so they
    agree to rounding, not bitwise)."""
    from paper_2306_15678_amd.march import plan_variants
    inst, u0, target = _adjoint_variant_case(4096)
    n_row, n_col = plan_variants(4096, 32)
    p = _prop([inst], 32, max_steps=inst.n_steps, ckpt_every=2)
    p.gen_screens()
    res = {}
    combos = [(r, 0) for r in range(n_row)] + [(0, c) for c in range(1, n_col)]
    for r, c in combos:
        p.select_plan(4096, r, c)
        p.select_adjoint_plan(4096, -1, -1)
        res[(r, c)] = _fwd_adj(p, inst, u0, target)
    l0, g0, t0 = res[(0, 0)]
    for key in combos[1:]:
        loss, gg, gt = res[key]
        lerr = abs(loss / l0 - 1)
        ferr = M.rel_l2(gg, g0)
        terr = float(np.max(np.abs(gt - t0)) / np.max(np.abs(t0)))
        _report(f"adjoint variants n=4096 {key} vs (0, 0)", loss=lerr, g_u0=ferr, g_theta=terr)
        assert lerr < 1e-5 and ferr < 1e-5 and terr < 1e-5, key
    # pipelined against the plain kernels of the same radices and threads:
    # rows 6, 7 against row 1; column 6 against column 1, column 7 against 0
    for key, ref in (((6, 0), (1, 0)), ((7, 0), (1, 0)), ((0, 6), (0, 1)), ((0, 7), (0, 0))):
        loss, gg, gt = res[key]
        ferr = M.rel_l2(gg, res[ref][1])
        terr = float(np.max(np.abs(gt - res[ref][2])) / np.max(np.abs(res[ref][2])))
        _report(f"pipelined variants {key} vs plain {ref}", g_u0=ferr, g_theta=terr,
                bitwise=bool(np.array_equal(gg, res[ref][1])))
        assert ferr < 1e-5 and terr < 1e-5, key


def test_pipelined_rows_batch_equals_each_beam_alone():
    """Two 2048^2 beams with different z steps (so different propagators) in
    one context: a persistent row or column workgroup takes lines of both
    beams in turn and reloads the propagator when the beam changes.  Forward + adjoint of
    each beam equals that beam in a context of its own, bitwise."""
    base, u0, target = _adjoint_variant_case(2048)
    other = dataclasses.replace(base, dz=0.007, seed=base.seed + 1)
    u1 = W.initial_field(other)
    pair = _prop([base, other], 32, max_steps=3, ckpt_every=2)
    pair.gen_screens()
    pair.select_plan(2048, 2, 2)
    for b, (inst, u) in enumerate(((base, u0), (other, u1))):
        pair.set_field(b, u)
        pair.set_theta(b, inst.theta)
    pair.forward_record(3)
    pair.fluence_loss(0, target)
    pair.fluence_loss(1, target)
    pair.backward()
    for b, (inst, u) in enumerate(((base, u0), (other, u1))):
        one = _prop([inst], 32, max_steps=3, ckpt_every=2)
        one.gen_screens()
        one.select_plan(2048, 2, 2)
        _fwd_adj(one, inst, u, target)
        assert np.array_equal(pair.grad_field(b), one.grad_field(0)), b
        assert np.array_equal(pair.grad_theta(b), one.grad_theta(0)), b


def test_headline_variants_batch_equals_each_beam_alone():
    """Two 4096^2 beams with different z steps in one context with the
    tile variants the tuner picks for the 4096^2 headline (row 8: twiddles
    in LDS; column 10: exchange through half the tile; also as the adjoint
    passes): each workgroup reads its own beam's tables, so forward +
    adjoint of each beam equals that beam in a context of its own,
    bitwise."""
    base, u0, target = _adjoint_variant_case(4096)
    other = dataclasses.replace(base, dz=base.dz * 0.7, seed=base.seed + 1)
    u1 = W.initial_field(other)
    pair = _prop([base, other], 32, max_steps=3, ckpt_every=2)
    pair.gen_screens()
    pair.select_plan(4096, 8, 10)
    pair.select_adjoint_plan(4096, 8, 10)
    for b, (inst, u) in enumerate(((base, u0), (other, u1))):
        pair.set_field(b, u)
        pair.set_theta(b, inst.theta)
    pair.forward_record(3)
    pair.fluence_loss(0, target)
    pair.fluence_loss(1, target)
    pair.backward()
    for b, (inst, u) in enumerate(((base, u0), (other, u1))):
        one = _prop([inst], 32, max_steps=3, ckpt_every=2)
        one.gen_screens()
        one.select_plan(4096, 8, 10)
        one.select_adjoint_plan(4096, 8, 10)
        _fwd_adj(one, inst, u, target)
        assert np.array_equal(pair.grad_field(b), one.grad_field(0)), b
        assert np.array_equal(pair.grad_theta(b), one.grad_theta(0)), b
        one.close()
    pair.close()


# ---------------------------------------------------------- config 3
# 64 uneven beams (n in {256, 512, 768, 1024}) with 20 Kolmogorov screens
# each, marched together in one context.  Checked on one beam of each size
# (indices 0, 1, 5, 10) over the first 100 steps (one screen, after step 49).
# Floors at step 100 (tests/golden/floor_c3_<beam>.json, oracle-only script):
#   beam  n     FP32 floor (max of peer / per-step)   FP64 per-step floor
#   0     1024  2.8e-5                                9.9e-15
#   1     768   4.8e-5                                2.7e-14
#   5     512   3.1e-5                                1.7e-14
#   10    256   5.7e-3 (185 P_cr: unstable by step 100) 7.7e-12
# Tolerance: FP32 5x, FP64 10x the floor.
C3_BEAMS = {0: (1.4e-4, 1e-13), 1: (2.4e-4, 2.7e-13), 5: (1.6e-4, 1.7e-13),
            10: (2.9e-2, 7.7e-11)}


@pytest.fixture(scope="module")
def c3_oracle():
    insts = W.config3()
    out = {}
    for b in C3_BEAMS:
        scr = T.instance_screens(insts[b])
        out[b] = (M.march(W.initial_field(insts[b]), insts[b], n_steps=100, screens=scr).field,
                  scr)
    return insts, out


def test_config3_screens_match_oracle(c3_oracle):
    insts, ref = c3_oracle
    p = _prop(insts, 32)
    p.gen_screens()
    for b in C3_BEAMS:
        steps = insts[b].screen_steps()
        for s in range(insts[b].n_screens):
            want = ref[b][1][steps[s]]
            got = p.screen(b, s)
            err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
            assert err < 2e-6, (b, s, err)


@pytest.mark.parametrize("precision", [32, 64])
def test_config3_batched_march_matches_oracle(c3_oracle, precision):
    insts, ref = c3_oracle
    p = _prop(insts, precision)
    p.gen_screens()
    for b, inst in enumerate(insts):
        p.set_field(b, W.initial_field(inst))
    p.propagate(100)
    for b, tol in C3_BEAMS.items():
        got = p.field(b)
        err = M.rel_l2(got, ref[b][0])
        emax = _maxrel(got, ref[b][0])
        _report(f"c3 beam {b} n={insts[b].n} fp{precision}", field=err, field_max=emax)
        t = tol[0] if precision == 32 else tol[1]
        assert err < t and emax < MAX_OVER_L2 * t, (b, err, emax)


def test_config3_batch_equals_each_beam_alone():
    insts = W.config3()
    p = _prop(insts, 32)
    p.gen_screens()
    for b, inst in enumerate(insts):
        p.set_field(b, W.initial_field(inst))
    p.propagate(100)
    for b in C3_BEAMS:
        q = _prop([insts[b]], 32)
        q.gen_screens()
        q.set_field(0, W.initial_field(insts[b]))
        q.propagate(100)
        assert np.array_equal(p.field(b), q.field(0)), b


# ---------------------------------------------------------- config 4
# Sparse 256^2 beam with the ansatz screen, 500 steps over 3 m, loss =
# fluence mismatch, adjoint with a checkpoint every 50 steps.  Parity of the
# gradient uses a target that comes from the input module (a dense-grid
# reference computed by the library must not feed the oracle).
def _c4():
    inst = W.config4_sparse()
    return inst, W.initial_field(inst), W.synthetic_target(inst, 44)


@pytest.fixture(scope="module")
def c4_oracle():
    inst, u0, target = _c4()
    return {m: M.gradient(u0, inst, n_steps=m, cotangent=lambda u: M.fluence_loss(u, target))
            for m in (100, 500)}


# Gradient floors (tests/golden/floor_c4.json, "gradient": loss, dL/dU0,
# dL/dtheta against the FP64 oracle gradient):
#             FP64 (input 2^-53)             FP32 peer (complex64, autodiff)
#   100 steps 7.1e-15 5.0e-14 6.4e-14         1.3e-4 1.1e-3 1.4e-3
#   500 steps 8.5e-12 1.1e-6  4.1e-10         1.6    4.6e2  3.5e1
# The sparse beam collapses chaotically (the ansatz at theta0 only mimics
# plasma arrest for x <= 1); FP32 gradients decorrelate after ~200 steps,
# so FP32 parity is stated at 100 steps and only reported at 500.  FP64
# tolerance: 10x the floor at 100 steps, 100x at 500 (the input floor omits
# per-step rounding, which over 500 chaotic steps adds one to two decades).
C4_TOL = {(64, 100): (7.1e-14, 5.0e-13, 6.4e-13), (64, 500): (8.5e-10, 1.1e-4, 4.1e-8),
          (32, 100): (6.5e-4, 5.5e-3, 7.0e-3)}


@pytest.mark.parametrize("precision,steps", [(64, 100), (64, 500), (32, 100), (32, 500)])
def test_config4_gradient_matches_oracle(c4_oracle, precision, steps):
    inst, u0, target = _c4()
    loss, g_u0, g_th = c4_oracle[steps]
    p = _prop([inst], precision, max_steps=steps, ckpt_every=50)
    p.set_field(0, u0)
    p.set_theta(0, inst.theta)
    p.forward_record(steps)
    gl = p.fluence_loss(0, target)
    p.backward()
    gu, gt = p.grad_field(0), p.grad_theta(0)
    lerr = abs(gl / loss - 1)
    ferr = M.rel_l2(gu, g_u0)
    terr = float(np.max(np.abs(gt - g_th)) / np.max(np.abs(g_th)))
    _report(f"c4 grad fp{precision} steps={steps}", loss=lerr, g_u0=ferr, g_theta=terr)
    assert np.isfinite(gl) and np.all(np.isfinite(gt)) and np.all(np.isfinite(gu))
    tol = C4_TOL.get((precision, steps))
    if tol is not None:
        assert lerr < tol[0] and ferr < tol[1] and terr < tol[2]


# R20 for config 4 in complex64: the input floor in32 (two FP64 marches
# whose inputs differ by 2^-24) is 7.0e-8, 2.9e-5, 4.6e-3, 3.8e-2, 7.6e-2
# at steps 100..500, so the largest sampled z with delta_32 <= 1e-3 is step
# 200 (1.2 m of 3 m).  Field and fluence parity are stated there, at 5x the
# largest FP32 floor of that step (peer32 6.1e-3 field / 6.7e-3 fluence;
# step32 1.1e-3 / 1.2e-3), and at step 100 (peer32 4.1e-5 / 9.5e-5).  At
# the full 500 steps the FP32 march is past the chaotic divergence (every
# FP32 floor is O(1)): no parity is claimed there; the power of both
# marches is reported (theta0's imaginary part is a gain at small x, so
# the power is not monotone) and the FP32 march must stay finite.
C4_FWD32_TOL = {100: (2.1e-4, 4.8e-4), 200: (3.1e-2, 3.4e-2)}


def test_config4_fp32_forward_at_the_r20_horizon():
    inst, u0, _ = _c4()
    p = _prop([inst], 32)
    p.set_field(0, u0)
    p.set_theta(0, inst.theta)
    u, done = u0, 0
    for stop, (tf, tw) in sorted(C4_FWD32_TOL.items()):
        ref = M.march(u, inst, n_steps=stop - done)
        u, done = ref.field, stop
        p.propagate(ref.power.size)
        got = p.field(0)
        err = M.rel_l2(got, ref.field)
        ferr = M.rel_l2(np.abs(got) ** 2, np.abs(ref.field) ** 2)
        _report(f"c4 fp32 forward step {stop}", field=err, fluence=ferr,
                field_max=_maxrel(got, ref.field))
        assert err < tf and ferr < tw
    ref = M.march(u, inst, n_steps=inst.n_steps - done)
    p.propagate(inst.n_steps - done)
    pw, _ = p.diag(0, inst.n_steps - done)
    perr = float(np.max(np.abs(pw / ref.power - 1)))
    _report("c4 fp32 forward step 500 (past the R20 horizon)", power=perr,
            power_oracle=float(ref.power[-1] / ref.power[0]),
            power_fp32=float(pw[-1] / pw[0]))
    assert np.all(np.isfinite(pw)) and np.all(np.isfinite(p.field(0)))


def test_config4_gradient_matches_finite_differences():
    """Central differences of the library's own FP64 loss in theta and in
    random complex directions of U0 (h = 1e-6 relative), over the first 100
    steps.  Past the collapse (about step 150) the loss of this march varies
    on scales below h (the FP64 loss already differs from the oracle's by
    2e-10 at step 500), so differences there measure curvature, not the
    derivative; the adjoint at 500 steps is compared with the oracle's."""
    inst, u0, target = _c4()
    steps = 100
    p = _prop([inst], 64, max_steps=steps, ckpt_every=50)

    def loss(u, th):
        p.set_field(0, u)
        p.set_theta(0, th)
        p.forward_record(steps)
        return p.fluence_loss(0, target)

    th0 = np.array(inst.theta)
    loss(u0, th0)
    p.backward()
    g_th, g_u0 = p.grad_theta(0), p.grad_field(0)
    for q in (0, 3, 5, 7):
        h = 1e-6 * max(1.0, abs(th0[q]))
        e = np.zeros(8)
        e[q] = h
        fd = (loss(u0, th0 + e) - loss(u0, th0 - e)) / (2 * h)
        _report(f"c4 fd theta{q}", fd=fd, adj=float(g_th[q]))
        assert abs(fd - g_th[q]) <= 1e-5 * max(abs(fd), 1e-3 * np.max(np.abs(g_th)))
    rng = np.random.default_rng(3)
    for _ in range(2):
        d = rng.standard_normal(u0.shape) + 1j * rng.standard_normal(u0.shape)
        h = 1e-6 * np.abs(u0).max() / np.abs(d).max()
        fd = (loss(u0 + h * d, th0) - loss(u0 - h * d, th0)) / (2 * h)
        an = float(np.real(np.vdot(g_u0, d)))
        _report("c4 fd u0", fd=fd, adj=an)
        assert abs(fd - an) <= 1e-5 * abs(fd)


def _descends(run, th0, g, l0, steps=(1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9)):
    """Backtracking along -g: the first step size that lowers the loss, or
    None.  Any differentiable loss with a nonzero gradient decreases for a
    small enough step."""
    d = g / np.max(np.abs(g))
    for h in steps:
        if run(th0 - h * d) < l0:
            return h
    return None


def test_config4_dense_reference_workflow():
    """The full workflow: 2048^2 dense march (6000 steps, Kerr + MPA +
    plasma, complex64) on the GPU, 8x8 block mean onto the sparse grid, then
    the sparse model's loss and theta gradient against that target (FP64:
    the 500-step sparse march is chaotic enough that complex64 gradients
    are rounding noise, see the FP32 gradient floors above).  Checked by
    properties: block mean against numpy on the same fluence, power never
    increasing, finite loss and gradients, and -g a descent direction."""
    dense = W.config4_dense()
    pd = _prop([dense], 32)
    pd.set_field(0, W.initial_field(dense))
    pw = []
    for _ in range(dense.n_steps // 2000):
        pd.propagate(2000)
        pw += list(pd.diag(0, 2000)[0])
    pw = np.array(pw)
    assert len(pw) == dense.n_steps
    assert np.all(np.isfinite(pw)) and np.all(np.diff(pw) <= 1e-6 * pw[0])
    fl = pd.intensity(0, device=True)
    tgt = pd.block_mean(fl, 8)
    want = M.block_mean(fl.cpu().numpy(), 8)
    assert np.max(np.abs(tgt.cpu().numpy() - want)) <= 1e-12 * np.max(want)
    pd.close()
    inst, u0, _ = _c4()
    p = _prop([inst], 64, max_steps=inst.n_steps, ckpt_every=50)
    tgt = tgt.double()
    th0 = np.array(inst.theta)

    def run(th):
        p.set_field(0, u0)
        p.set_theta(0, th)
        p.forward_record(inst.n_steps)
        return p.fluence_loss(0, tgt)

    l0 = run(th0)
    p.backward()
    g = p.grad_theta(0)
    assert np.isfinite(l0) and np.all(np.isfinite(g)) and np.any(g != 0)
    h = _descends(run, th0, g, l0)
    _report("c4 workflow", loss0=l0, descent_step=h, power_end=float(pw[-1] / pw[0]))
    assert h is not None


# ---------------------------------------------------------- config 2
# The bench workload at full size: 1024^2, 2000 steps, the tuned tile
# variants.  Compared with the oracle's own samples of the same march
# (tests/golden/floor_c2.json, written by calibrate_floor.py c2 from the
# oracle alone): the field at 64 seeded points every 100 steps, power and
# peak intensity after every step, and 32x32-block fluence at 500, 1000,
# 1500 and 2000 steps.  Floors in the same file.  FP64: 10x the largest of
# the per-step and input floors and the independent complex128 peer (whose
# coherent table rounding dominates: 4e-13 at step 1000 against 3e-14 for
# the random per-step model), at every sample to the end.  FP32: the floor
# passes 1e-3 after step 1100, where the multifilament march turns chaotic,
# so FP32 field parity is stated up to step 1100 (5x the larger of the
# complex64 peer and the per-step floor) and the global diagnostics (block
# fluence, power, peak) to the end at 5x the peer's.
def _c2_ref():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "floor_c2.json")
    return json.load(open(path))


@pytest.mark.parametrize("precision", [64, 32])
def test_config2_full_size_against_oracle_samples(precision):
    from paper_2306_15678_amd.tune import tune
    d = _c2_ref()
    ref = d["reference"]
    pts = np.array(d["sample_points"])
    inst = W.config2()[0]
    p = _prop([inst], precision)
    tune(p, reps=5, use_cache=False)
    p.set_field(0, W.initial_field(inst))
    power, peak = [], []
    for k, m in enumerate(d["steps"]):
        p.propagate(100)
        pw, pk = p.diag(0, 100)
        power += list(pw)
        peak += list(pk)
        u = p.field(0)
        want = np.array(ref["field_re"][str(m)]) + 1j * np.array(ref["field_im"][str(m)])
        got = u[pts[:, 0], pts[:, 1]]
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        emax = _maxrel(got, want)
        if str(m) in ref["block_fluence"]:
            bf = np.array(ref["block_fluence"][str(m)])
            gb = M.block_mean(np.abs(u) ** 2, inst.n // bf.shape[0])
            berr = float(np.linalg.norm(gb - bf) / np.linalg.norm(bf))
            _report(f"c2 fp{precision} step {m}", samples=err, samples_max=emax,
                    block_fluence=berr)
            if precision == 32:
                assert berr < 5 * d["peer32"]["block_fluence"][k], (m, berr)
            else:
                assert berr < 10 * d["peer64"]["block_fluence"][k], (m, berr)
        if precision == 64:
            floor = max(d["step64"]["field"][k], d["in64"]["field"][k], d["peer64"]["field"][k])
            assert err < 10 * floor and emax < MAX_OVER_L2 * 10 * floor, (m, err, emax, floor)
        elif m <= 1100:
            floor = max(d["peer32"]["field"][k], d["step32"]["field"][k])
            assert err < 5 * floor and emax < MAX_OVER_L2 * 5 * floor, (m, err, emax, floor)
    perr = np.abs(np.array(power) / np.array(ref["power"]) - 1)
    kerr = np.abs(np.array(peak) / np.array(ref["peak"]) - 1)
    _report(f"c2 fp{precision} diag", power_max=float(perr.max()), power_end=float(perr[-1]),
            peak_1100=float(kerr[:1100].max()), peak_end=float(kerr[-1]))
    # largest relative power / peak difference over steps 1..m, against the
    # same for the independent peer of this precision (10x FP64, 5x FP32)
    peer, f = ("peer64", 10) if precision == 64 else ("peer32", 5)
    for k, m in enumerate(d["steps"]):
        assert perr[:m].max() < f * d[peer]["power"][k], (m, perr[:m].max())
        assert kerr[:m].max() < f * d[peer]["peak"][k], (m, kerr[:m].max())


# ---------------------------------------------------------- config 5
# 4096^2, 2.5 cm beam at 1000 P_cr, all screen terms and 50 Kolmogorov
# screens over 1 km (5000 steps).  The FP64 oracle needs seconds per step at
# this size, so parity is checked on the first 10 steps at full size (and on
# the first screen pair); the full forward + adjoint march is checked by
# properties that hold at any length.
# Floors at step 10 (tests/golden/floor_c5.json): FP32 peer 1.3e-6, per-step
# FP32 1.4e-6 -> tolerance 5x = 7e-6.  FP64: the oracle evaluates the
# diffraction factor exp(-i k^2 dz / 2k0) without reducing the phase, which
# reaches 146 rad at the Nyquist mode of this grid, so its own error is up to
# 146 x 2^-53 = 1.6e-14 per step (1.6e-13 over 10 steps; the library reduces
# the phase modulo 2 pi in FP64 first) -> tolerance 10x that bound.
C5_TOL = {64: 1.6e-12, 32: 7e-6}


@pytest.fixture(scope="module")
def c5_oracle():
    inst = W.config5()[0]
    u0 = W.initial_field(inst)
    return inst, u0, M.march(u0, inst, n_steps=10).field


@pytest.mark.parametrize("precision", [64, 32])
def test_config5_prefix_matches_oracle(c5_oracle, precision):
    inst, u0, ref = c5_oracle
    p = _prop([inst], precision)
    p.set_field(0, u0)
    p.propagate(10)
    got = p.field(0)
    err = M.rel_l2(got, ref)
    emax = _maxrel(got, ref)
    _report(f"c5 10 steps fp{precision}", field=err, field_max=emax)
    assert err < C5_TOL[precision] and emax < MAX_OVER_L2 * C5_TOL[precision]


def test_config5_first_screens_match_oracle():
    inst = W.config5()[0]
    k0 = 2 * math.pi / inst.medium.wavelength
    amp = T.kolmogorov_amplitude(inst.n, inst.length,
                                 T.fried_parameter(k0, inst.cn2, inst.screen_dz))
    re, im = T.screen_pair(inst.n, inst.length, amp, inst.seed, 0)
    from paper_2306_15678_amd.march import plan_variants
    p = _prop([inst], 32)
    # the column inverse transform of every column variant
    for v in range(plan_variants(inst.n, 32)[1]):
        p.select_plan(inst.n, 0, v)
        p.gen_screens()
        for s, want in ((0, re), (1, im)):
            got = p.screen(0, s)
            err = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
            _report(f"c5 screen {s} column variant {v}", maxrel=err)
            assert err < 2e-6, v


def test_config5_gradient_prefix_matches_oracle():
    """The FP64 adjoint at full size (4096^2, all screen terms, seeded
    theta) over the first 3 steps against the oracle's gradient."""
    inst = W.config5()[0]
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    theta = 0.05 * W.random_theta(56, 1.0)
    steps = 3
    # no screen falls in the first 3 steps (the first is after step 99)
    l_ref, g_ref, t_ref = M.gradient(u0, inst, n_steps=steps, theta=theta,
                                     cotangent=lambda u: M.fluence_loss(u, target))
    p = _prop([inst], 64, max_steps=steps, ckpt_every=steps)
    p.set_field(0, u0)
    p.set_theta(0, theta)
    p.forward_record(steps)
    gl = p.fluence_loss(0, target)
    p.backward()
    gu, gt = p.grad_field(0), p.grad_theta(0)
    lerr = abs(gl / l_ref - 1)
    ferr = M.rel_l2(gu, g_ref)
    terr = float(np.max(np.abs(gt - t_ref)) / np.max(np.abs(t_ref)))
    _report("c5 grad fp64 steps=3", loss=lerr, g_u0=ferr, g_theta=terr)
    assert lerr < C5_TOL[64] and ferr < C5_TOL[64] and terr < C5_TOL[64]


def _absorbing_theta(seed):
    """Seeded ansatz coefficients whose imaginary part is nonnegative, so the
    ansatz only absorbs: (0.05 N(0,1) phase, 0.05 |N(0,1)| absorption)."""
    th = 0.05 * W.random_theta(seed, 1.0)
    th[4:] = np.abs(th[4:])
    return th


def test_nonfinite_theta_gradient_is_reported():
    """With gain coefficients (negative imaginary theta) the linearised
    4096^2 march grows by about e^1.45 per step (the Kerr phase per step is
    25 rad at I = I_a), so the complex64 adjoint overflows within 200 steps;
    ssfm_get_grad_theta reports SSFM_ENONFINITE instead of returning NaN
    silently.  Only the arithmetic overflows: every kernel runs normally."""
    from paper_2306_15678_amd._lib import ENONFINITE, SsfmError
    inst = W.config5()[0]
    theta = 0.05 * W.random_theta(55, 1.0)
    assert np.any(theta[4:] < 0)
    p = _prop([inst], 32, max_steps=200, ckpt_every=71)
    p.gen_screens()
    p.set_field(0, W.initial_field(inst))
    p.set_theta(0, theta)
    p.forward_record(200)
    p.set_cotangent(0, W.random_field_like(inst.n, 7, 1.0))
    p.backward()
    with pytest.raises(SsfmError) as e:
        p.grad_theta(0)
    assert e.value.status == ENONFINITE


def test_config5_full_forward_adjoint_properties():
    """5000 steps, checkpoint every 71 steps (about sqrt(5000): 71 + 2 x 70
    fields), twin experiment against the fluence of a run with a seeded,
    absorbing theta_ref.  At theta_ref the loss and the gradients are at rounding
    level.  At theta = 0: finite loss and gradients, power never increasing, and
    gradients bitwise independent of the checkpoint interval (a recomputed
    segment repeats the recorded march exactly).  After 1 km the complex64
    march is chaotic (loss ~1 against its own twin), so no descent claim is
    made here; descent and finite differences are checked on shorter
    marches."""
    import torch
    inst = W.config5()[0]
    u0 = W.initial_field(inst)
    theta_ref = _absorbing_theta(55)
    th0 = np.zeros(8)
    grads = {}
    for ckpt in (71, 100):
        p = _prop([inst], 32, max_steps=inst.n_steps, ckpt_every=ckpt)
        p.gen_screens()
        p.set_field(0, u0)
        p.set_theta(0, theta_ref)
        p.propagate(inst.n_steps)
        target = p.intensity(0, device=True)

        def run(th):
            p.set_field(0, u0)
            p.set_theta(0, th)
            p.forward_record(inst.n_steps)
            return p.fluence_loss(0, target)

        if ckpt == 71:
            # the target is read out by the field store and the loss by the
            # seed kernel: the same FP64 intensity up to operation order
            l_ref = run(theta_ref)
            p.backward()
            g_ref = float(np.max(np.abs(p.grad_theta(0))))
            gu_ref = float(p.grad_field(0, device=True).abs().max())
        l0 = run(th0)
        pw, _ = p.diag(0, inst.n_steps)
        p.backward()
        g = p.grad_theta(0)
        gu = p.grad_field(0, device=True)
        assert np.isfinite(l0) and l0 > 0 and np.all(np.isfinite(g)) and np.any(g != 0)
        assert bool(gu.isfinite().all())
        assert np.all(np.diff(pw) <= 1e-6 * pw[0])
        grads[ckpt] = (l0, g, gu.cpu())
        _report(f"c5 fwd+adj ckpt={ckpt}", loss0=l0, power_end=float(pw[-1] / pw[0]))
        p.close()
        del p
        torch.cuda.empty_cache()
    # at theta_ref the residual is rounding of the intensity (~1e-16), and
    # the gradients are linear in it
    _report("c5 twin", loss=l_ref, g_theta=g_ref, g_u0=gu_ref)
    assert l_ref < 1e-26
    assert g_ref <= 1e-10 * np.max(np.abs(grads[71][1]))
    assert gu_ref <= 1e-10 * float(grads[71][2].abs().max())
    assert grads[71][0] == grads[100][0]
    assert np.array_equal(grads[71][1], grads[100][1])
    assert torch.equal(grads[71][2], grads[100][2])


# ------------------------------------------------------------ pass timing
@pytest.mark.parametrize("graphs", [True, False])
def test_pass_timing_samples(graphs):
    """Sampled in-march pass timing: the expected number of samples (steps
    s with s % 10 == 5 of the last forward march), positive durations of the
    order of the isolated pass timing, and fields bitwise identical to a run
    without sampling."""
    inst = W.config2()[0]
    u0 = W.initial_field(inst)
    out = {}
    for every in (0, 10):
        p = _prop([inst], 32, max_steps=60, ckpt_every=20)
        p.use_graphs(graphs)
        p.set_pass_timing(every)
        p.set_field(0, u0)
        p.propagate(37)              # steps 0..36: samples at 5, 15, 25, 35
        r, c, n = p.pass_times()
        assert n == (4 if every else 0)
        if every:
            iso_r, iso_c, _, _ = p.time_passes(reps=20)
            _report(f"pass timing graphs={graphs}", row=r, col=c, iso_row=iso_r, iso_col=iso_c)
            assert 0 < r < 3 * iso_r and 0 < c < 3 * iso_c
            p.forward_record(40)      # steps 37..76: samples at 45, 55, 65, 75
            assert p.pass_times()[2] == 4
        else:
            p.forward_record(40)
        out[every] = p.field(0)
        p.close()
    assert np.array_equal(out[0], out[10])


# ------------------------------------------------ step-spectrum screens
def _step_instance():
    # 60 steps: the first screen (after step 49) acts, and the 185 P_cr beam
    # is still far from its collapse (per-step FP64 floor 2.4e-14 here; at
    # 120 steps its peak has grown 42x and the floor is 4e-10)
    inst = dataclasses.replace([b for b in W.config3() if b.n == 256][0], n_steps=60)
    val = 1.0 / (inst.n * (inst.length / inst.n))
    k_h = 2.0 * math.pi * (5 * val)      # exactly on the |m| = 5 ring of modes
    return inst, (4e-3, k_h)


def test_step_spectrum_screens_match_oracle():
    inst, step = _step_instance()
    want = T.instance_screens(inst, step_spectrum=step)
    p = _prop([inst], 32)
    p.set_screen_spectrum(0, step)
    p.gen_screens()
    steps = sorted(want)
    amp = T.step_amplitude(inst.n, inst.length, *step)
    for s_idx, st in enumerate(steps[:4]):
        got = p.screen(0, s_idx)
        err = float(np.max(np.abs(got - want[st])) / np.max(np.abs(want[st])))
        _report(f"step spectrum screen {s_idx}", maxrel=err)
        assert err < 2e-6, (s_idx, err)
    re, im = p.screen(0, 0), p.screen(0, 1)
    spec = np.fft.fft2(re + 1j * im)
    assert np.max(np.abs(spec[amp == 0])) < 1e-5 * np.max(np.abs(spec))
    p.close()


def test_step_spectrum_march_matches_oracle():
    inst, step = _step_instance()
    screens = T.instance_screens(inst, step_spectrum=step)
    u0 = W.initial_field(inst)
    ref = M.march(u0, inst, screens=screens).field
    p = _prop([inst], 64)
    p.set_screen_spectrum(0, step)
    p.gen_screens()
    p.set_field(0, u0)
    p.propagate(inst.n_steps)
    err = M.rel_l2(p.field(0), ref)
    _report("step spectrum march fp64", field=err)
    assert err < 10 * 2.4e-14  # 10x the per-step FP64 floor of this march
    p.close()


def test_many_small_chunks_equal_one_march():
    """150 one-step propagates (graph mode: one captured graph per start
    step, so the bounded graph cache is emptied on the way) give the field
    of one 150-step propagate bitwise."""
    inst = W.config1()[0]
    u0 = W.initial_field(inst)
    p = _prop([inst], 32)
    p.set_field(0, u0)
    p.propagate(150)
    one = p.field(0)
    p.set_field(0, u0)
    for _ in range(150):
        p.propagate(1)
    assert np.array_equal(p.field(0), one)
    p.close()
