"""Throughput of the split-step march on one MI355X (grid-point . steps / s).

Headline workload: the large-aperture beam on a 4096 x 4096 grid (2.5 cm,
1000 P_cr, Kerr + multiphoton absorption + saturating plasma + the ansatz
screen, 50 Kolmogorov turbulence screens over 1 km), 5000 z steps of 20 cm,
complex64 with FP64 reductions.  One bench step is the whole differentiable
march: the recorded forward march (checkpoints every M steps, M sized so the
checkpoints and two segment banks fit the device), the fluence-mismatch loss
against a synthetic target, and the exact adjoint back to the input field
(each segment recomputed from its checkpoint beside the adjoint of the
next).  Grid-point . steps count each z step once.  The timed steps run
unsampled, every march in its captured graphs.

A separate, untimed run of the same step samples the pass kernels with HIP
events on the library's stream (forward passes of the record, adjoint
passes of the first checkpoint segment): the roofline names the kernel with
the largest estimated total time in the march and divides its algorithmic
bytes per launch by its mean duration.

The JSON line also carries the same march with the complex128 kernels, the
whole-march HBM fraction, the extra workloads (the 1024^2 multifilament
beam forward + adjoint, the 64-beam batch forward and forward + adjoint,
one genetic-search generation, the scheme variants, the paper's beam
diagnostics) and the FP64 CPU oracle timed on a bounded sample of the
headline workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extra]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid-point·steps/s SSFM fwd+adjoint, FP32 vs FP64, at stated L2 error"
UNIT = "grid-point·steps/s"
# sampled steps: s % SAMPLE_EVERY == SAMPLE_EVERY / 2.  The turbulence screens
# of the headline beam act on the row pass of steps 100 k + 50 (forward) and
# on the adjoint row pass of the same steps, whose residues mod 8 are 2 and
# 6: the samples are the typical, screen-free step.
SAMPLE_EVERY = 8
# z steps at which the complex64 and complex128 marches are compared, and
# the length of the short forward+adjoint compared within the horizon
SNAP_STEPS = (5, 10, 20, 50, 100, 150, 200, 300, 500, 1000, 2000, 5000)
SHORT_STEPS = 100
# device memory left outside the headline march's workspace (torch's own
# allocations, the runtime, the timing events)
WORKSPACE_RESERVE = 20 * 2 ** 30
# algorithmic HBM bytes per grid point of one launch (complex64): a pass
# reads and writes the field; the adjoint row pass also reads the stored
# pre-screen field
PASS_BYTES = {"row_fwd": 16, "col_fwd": 16, "col_adj": 16, "row_adj": 24}


def _desc_list(insts):
    from paper_2306_15678_amd.march import desc_of
    return [desc_of(i) for i in insts]


def _timed(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def _say(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _ckpt_plan(n_steps, m):
    """(segments, recomputed steps) of a recorded march of n_steps with a
    checkpoint every m steps (m >= n_steps: everything stored)."""
    if m >= n_steps:
        return 1, 0
    seg = -(-n_steps // m)
    return seg, n_steps - seg


# ------------------------------------------------------------ headline
def run_headline(args):
    """Config 5 forward + adjoint, FP32 timed unsampled, then one sampled
    (untimed) step for the pass kernels, then the complex128 form."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator, checkpoint_plan
    from paper_2306_15678_amd.tune import tune

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(0)
    inst = W.config5()[0]
    n, z_steps = inst.n, inst.n_steps
    u0_d = torch.from_numpy(W.initial_field(inst)).to(dev)
    tgt_d = torch.from_numpy(W.synthetic_target(inst, 5)).to(dev)
    gp_steps = float(n) * n * z_steps
    out = {}

    def make(precision):
        # checkpoints every M steps, the last K segments kept whole: the
        # layout that fits the free HBM less WORKSPACE_RESERVE and
        # recomputes the fewest steps (or plain checkpointing every
        # --ckpt-every steps)
        if args.ckpt_every:
            m, k = args.ckpt_every, 0
            rec = _ckpt_plan(z_steps, m)[1]
        else:
            budget = torch.cuda.mem_get_info()[0] - WORKSPACE_RESERVE
            m, k, rec = checkpoint_plan(_desc_list([inst]), precision, z_steps, budget)
        p = Propagator(_desc_list([inst]), precision=precision, max_steps=z_steps,
                       ckpt_every=m, stored_segments=k, device=dev)
        tuned = tune(p, reps=10, use_cache=False)[n]
        p.gen_screens()
        p.set_theta(0, inst.theta)
        return p, {"ckpt_every": m, "stored_segments": k, "recomputed_steps": rec}, tuned

    def fwd_adj(p, steps=z_steps):
        def go():
            p.set_field(0, u0_d)
            p.forward_record(steps)
            go.loss = p.fluence_loss(0, tgt_d)
            p.backward()
        return go

    def fluence_track(p):
        """Fluence |U|^2 at the SNAP_STEPS of a forward march from U_0 (host
        float64), then the loss and theta gradient of a SHORT_STEPS forward
        + adjoint: for the complex64 / complex128 comparison."""
        p.set_field(0, u0_d)
        out, done = [], 0
        for z in SNAP_STEPS:
            p.propagate(z - done)
            done = z
            out.append(p.intensity(0))
        go = fwd_adj(p, SHORT_STEPS)
        go()
        return out, go.loss, p.grad_theta(0)

    p, ck, tuned = make(32)
    _say(f"headline fp32: 4096^2 x {z_steps} steps, checkpoint every {ck['ckpt_every']}, "
         f"last {ck['stored_segments']} segments kept, {ck['recomputed_steps']} steps "
         f"recomputed, workspace {p.ws_bytes / 2**30:.1f} GiB")
    t = _timed(fwd_adj(p), args.steps, args.warmup, p.synchronize)
    out["fp32"] = {"s_per_step": t, "value": gp_steps / t, **ck,
                   "workspace_GiB": p.ws_bytes / 2 ** 30, "tune": tuned}
    _say(f"headline fp32: {t:.3f} s per step, {gp_steps / t:.3e} {UNIT}")
    # the same step sampled (untimed): pass kernels bracketed by events
    p.set_pass_timing(SAMPLE_EVERY)
    go = fwd_adj(p)
    go()
    p.synchronize()
    out["fp32"]["loss"] = go.loss
    out["fp32"]["grad_theta"] = p.grad_theta(0)
    ms_row, ms_col, n_fwd = p.pass_times()
    ms_cadj, ms_radj, n_adj = p.adjoint_pass_times()
    p.set_pass_timing(0)
    out["passes"] = {"row_fwd": ms_row, "col_fwd": ms_col, "col_adj": ms_cadj,
                     "row_adj": ms_radj, "samples_fwd": n_fwd, "samples_adj": n_adj}
    # forward only, same context
    def fwd():
        p.set_field(0, u0_d)
        p.propagate(z_steps)
    tf = _timed(fwd, 1, 1, p.synchronize)
    out["fwd"] = {"s_per_step": tf, "value": gp_steps / tf}
    pw, pk = p.diag(0, z_steps)
    out["power_end_over_start"] = float(pw[-1] / pw[0])
    out["power_monotone"] = bool(np.all(np.diff(pw) <= 1e-6 * pw[0]))
    flu32 = None if args.no_fp64 else fluence_track(p)
    p.close()
    del p, go  # go's closure holds the context (and its workspace) too
    torch.cuda.empty_cache()
    if not args.no_fp64:
        free, total = torch.cuda.mem_get_info()
        _say(f"free device memory {free / 2**30:.1f} of {total / 2**30:.1f} GiB "
             f"(torch holds {torch.cuda.memory_allocated() / 2**30:.2f} GiB)")
        q, ck64, tuned64 = make(64)
        _say(f"headline fp64: checkpoint every {ck64['ckpt_every']}, last "
             f"{ck64['stored_segments']} segments kept")
        go64 = fwd_adj(q)
        t64 = _timed(go64, 1, 1, q.synchronize)
        out["fp64"] = {"s_per_step": t64, "value": gp_steps / t64, **ck64,
                       "workspace_GiB": q.ws_bytes / 2 ** 30, "tune": tuned64}
        g64 = q.grad_theta(0)
        g32 = out["fp32"]["grad_theta"]
        flu64, loss64s, g64s = fluence_track(q)
        flu32, loss32s, g32s = flu32
        errs = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(flu32, flu64)]
        within = [z for z, e in zip(SNAP_STEPS, errs) if e <= 1e-3]
        out["fp32_vs_fp64"] = {
            "z_steps": list(SNAP_STEPS),
            "fluence_rel_l2": errs,
            "largest_z_steps_within_1e-3": max(within) if within else 0,
            f"loss_rel_{SHORT_STEPS}_steps": abs(loss32s / loss64s - 1),
            f"grad_theta_maxrel_{SHORT_STEPS}_steps":
                float(np.max(np.abs(g32s - g64s)) / np.max(np.abs(g64s))),
            "loss_rel_full": abs(out["fp32"]["loss"] / go64.loss - 1),
            "grad_theta_maxrel_full": float(np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))),
            "note": "complex64 march against the complex128 march of the same kernels (the "
                    "complex128 kernels match the FP64 oracle to 1e-11 on this beam over its "
                    "first steps): relative L2 of the fluence at each z, and loss / theta "
                    "gradient of a short and of the full forward+adjoint.  The beam "
                    "filaments (1000 P_cr); rounding differences grow with z, so past the "
                    "stated horizon the two precisions follow different (equally valid) "
                    "realisations of the chaotic march"}
        q.close()
        del q, go64
        torch.cuda.empty_cache()
    return out


def roofline(head, copy_peak):
    """Dominant kernel of the march (largest estimated total time) and its
    algorithmic bandwidth per launch."""
    import workloads as W
    inst = W.config5()[0]
    n2, z = float(inst.n) ** 2, inst.n_steps
    ps = head["passes"]
    recomputed = head["fp32"]["recomputed_steps"]
    launches = {"row_fwd": z + recomputed, "col_fwd": z + recomputed, "col_adj": z,
                "row_adj": z}
    total = {k: ps[k] * launches[k] for k in launches}
    dom = max(total, key=total.get)
    bytes_launch = PASS_BYTES[dom] * n2
    achieved = bytes_launch / (ps[dom] * 1e-3) / 1e9
    traffic = traffic_per_launch(dom)
    names = {"row_fwd": "forward row pass (pending screen fused)",
             "col_fwd": "forward column pass (FP64 power partials)",
             "col_adj": "adjoint column pass",
             "row_adj": "adjoint row pass (adjoint screen and theta partials fused)"}
    return {
        "bound": "hbm",
        "kernel": names[dom] + ", 4096^2 complex64",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_over_algorithmic": (traffic / bytes_launch) if traffic else None,
        "bytes_per_launch": bytes_launch,
        "ms_per_launch": ps[dom],
        "measured_copy_GBps": copy_peak,
        "frac_of_measured_copy": achieved / copy_peak,
        "est_total_ms_per_march": total,
        "timing": f"HIP events on the library stream around the passes of every "
                  f"{SAMPLE_EVERY}th step of a separate, untimed forward + adjoint step "
                  f"({ps['samples_fwd']} forward and {ps['samples_adj']} adjoint samples; "
                  "adjoint samples from the first checkpoint segment, which runs without "
                  "a recompute beside it)",
    }


def traffic_per_launch(kind):
    """HBM bytes per launch of pass `kind` on the 4096^2 grid, from the
    committed FETCH_SIZE / WRITE_SIZE summary (each counter scaled by its
    reading for a plain copy kernel of known size); None when absent or
    taken on other kernel sources."""
    from paper_2306_15678_amd.passprof import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "traffic_c5_4096.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    c = d["copy_kernel"]
    e = d.get("kernels", {}).get(kind)
    if not e:
        return None
    return 1024.0 * (e["fetch_kib"] / c["fetch_scale"] + e["write_kib"] / c["write_scale"])


# ---------------------------------------------------------------- extras
def run_c2_fwd_adj(args):
    """The 1024^2 multifilament beam (2000 steps), forward + adjoint with
    the whole trajectory kept, complex64; parity against the oracle's
    stored samples of this march."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator, checkpoint_plan
    from paper_2306_15678_amd.tune import tune
    dev = torch.device("cuda", 0)
    inst = W.config2()[0]
    z = inst.n_steps
    m, k, _ = checkpoint_plan(_desc_list([inst]), 32, z)
    p = Propagator(_desc_list([inst]), precision=32, max_steps=z, ckpt_every=m,
                   stored_segments=k, device=dev)
    tune(p, reps=10, use_cache=False)
    u0_d = torch.from_numpy(W.initial_field(inst)).to(dev)
    tgt_d = torch.from_numpy(W.synthetic_target(inst, 2)).to(dev)

    def go():
        p.set_field(0, u0_d)
        p.forward_record(z)
        p.fluence_loss(0, tgt_d)
        p.backward()
    t = _timed(go, max(2, args.steps), 1, p.synchronize)
    p.set_field(0, u0_d)
    p.propagate(z)
    pw, pk = p.diag(0, z)
    par = parity_vs_stored(inst, pw, pk, p.intensity(0))
    diag = time_diagnostics(p, inst, args)
    p.close()
    gp = float(inst.n) ** 2 * z
    return {"workload": "multifilament beam, 1024x1024 complex64, Kerr+MPA+plasma, "
                        f"2000 z steps, forward+adjoint, checkpoint every {m}",
            "value": gp / t, "unit": UNIT, "ms_per_step": t * 1e3, "ckpt_every": m,
            "stored_segments": k,
            "parity": par, "diagnostics": diag}


def run_batched(args):
    """The 64 uneven beams (n in {256, 512, 768, 1024}, 20 screens each,
    2000 steps) in one context: forward march, and forward + adjoint with a
    fluence loss on every beam."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator, checkpoint_plan
    from paper_2306_15678_amd.tune import tune
    insts = W.config3()
    z = insts[0].n_steps
    gp = float(sum(i.n * i.n for i in insts)) * z
    m, k, _ = checkpoint_plan(_desc_list(insts), 32, z)
    p = Propagator(_desc_list(insts), precision=32, max_steps=z, ckpt_every=m,
                   stored_segments=k, device=torch.device("cuda", 0))
    tune(p, reps=10, use_cache=False)
    p.gen_screens()
    fields = [torch.from_numpy(W.initial_field(i)).to("cuda") for i in insts]
    targets = [torch.from_numpy(W.synthetic_target(i, 300 + b)).to("cuda")
               for b, i in enumerate(insts)]

    def set_all():
        for b, u in enumerate(fields):
            p.set_field(b, u)

    def fwd():
        set_all()
        p.propagate(z)

    def fwd_adj():
        set_all()
        p.forward_record(z)
        for b, tg in enumerate(targets):
            p.fluence_loss(b, tg)
        p.backward()

    tf = _timed(fwd, max(1, args.steps // 2), 1, p.synchronize)
    ta = _timed(fwd_adj, max(1, args.steps // 2), 1, p.synchronize)
    p.close()
    work = "64 beams, n in {256,512,768,1024}, 20 Kolmogorov screens each, " \
           "Kerr+MPA+plasma, 2000 z steps, complex64"
    return ({"workload": work + ", forward", "value": gp / tf, "unit": UNIT,
             "ms_per_march": tf * 1e3},
            {"workload": work + f", forward+adjoint (fluence loss on every beam), "
                                f"checkpoint every {m}, last {k} segments kept",
             "value": gp / ta, "unit": UNIT, "ms_per_step": ta * 1e3, "ckpt_every": m,
             "stored_segments": k})


FD_ITERS = 4


def run_schemes(args):
    """Scheme variants on the 1024^2 workload, complex64, forward: Strang
    splitting beside Lie (2000 steps); the finite-difference reference
    scheme (500 steps, FD_ITERS iterations per step); 3 subharmonic levels
    in the screen synthesis of the 64-beam batch."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator
    from paper_2306_15678_amd.tune import tune

    dev = torch.device("cuda", 0)
    inst = W.config2()[0]
    n = inst.n
    u0_d = torch.from_numpy(W.initial_field(inst)).to(dev)
    out = {}
    p = Propagator(_desc_list([inst]), precision=32, device=dev)
    tune(p, reps=10, use_cache=False)

    def fwd(steps):
        def go():
            p.set_field(0, u0_d)
            p.propagate(steps)
        return go

    reps = max(1, args.steps // 2)
    t_lie = _timed(fwd(inst.n_steps), reps, 1, p.synchronize)
    p.set_splitting(True)
    t_strang = _timed(fwd(inst.n_steps), reps, 1, p.synchronize)
    gp = float(n) * n * inst.n_steps
    out["strang_forward"] = {"z_steps": inst.n_steps, "value": gp / t_strang, "unit": UNIT,
                             "ms_per_march": t_strang * 1e3, "lie_ms_per_march": t_lie * 1e3}
    fd_steps = 500
    p.set_finite_difference(FD_ITERS)
    t_fd = _timed(fwd(fd_steps), reps, 1, p.synchronize)
    pw, _ = p.diag(0, fd_steps)
    field_bytes = 8.0 * n * n
    step_bytes = field_bytes * (2 * FD_ITERS + 3 * (FD_ITERS - 1) + 4)
    us_step = t_fd / fd_steps * 1e6
    out["fd_reference"] = {
        "workload": f"{n}x{n} complex64, Kerr+MPA+plasma, {fd_steps} z steps, "
                    f"{FD_ITERS} fixed-point iterations per step",
        "value": float(n) * n * fd_steps / t_fd, "unit": UNIT,
        "us_per_step": us_step, "launches_per_step": 2 * FD_ITERS,
        "bytes_per_step": step_bytes, "achieved_GBps": step_bytes / (us_step * 1e-6) / 1e9,
        "power_drift": float(abs(pw[-1] / pw[0] - 1))}
    p.close()
    del p
    torch.cuda.empty_cache()
    insts = W.config3()
    q = Propagator(_desc_list(insts), precision=32, device=dev)
    t0 = _timed(q.gen_screens, 3, 1, q.synchronize)
    for b in range(len(insts)):
        q.set_subharmonics(b, 3)
    t3 = _timed(q.gen_screens, 3, 1, q.synchronize)
    q.close()
    out["subharmonics"] = {"workload": "64 beams x 20 screens, n in 256..1024, 3 levels",
                           "gen_screens_ms": t0 * 1e3, "with_3_levels_ms": t3 * 1e3}
    return out


def time_diagnostics(p, inst, args):
    """The paper's beam diagnostics on the end fluence: hot-area count
    (regions above 1 % of the peak, periodic), the energy moment Q(1, 1),
    one effective-lens screen and its vector-Jacobian product, per call
    including the host synchronisation; the oracle's count beside it."""
    import torch
    from paper_2306_15678_amd.march import hot_areas_static, make_lens
    w = p.intensity(0, device=True)
    thr = 0.01 * float(w.max())
    reps = 5
    count = p.hot_areas(w, thr)
    t0 = time.perf_counter()
    for _ in range(reps):
        p.hot_areas(w, thr)
    t_hot = (time.perf_counter() - t0) / reps
    assert hot_areas_static(w, thr) == count
    t0 = time.perf_counter()
    for _ in range(reps):
        p.moment(w, inst.length, 1.0, 1)
    t_mom = (time.perf_counter() - t0) / reps
    peak = float(w.max())
    dx = inst.length / inst.n
    c2 = (0.3e-3) ** 3
    lens = make_lens(4 * dx * dx, 0.2 * peak, -2.0 * peak / c2, c2,
                     [(0.28e-3, 0.7, 2.0e4, 0.0)], [(0.28e-3, 0.05, 1.0e4, 0.0)])
    p.apply_lens(0, lens)
    t0 = time.perf_counter()
    for _ in range(reps):
        p.apply_lens(0, lens)
    t_lens = (time.perf_counter() - t0) / reps
    u = p.field(0, device=True)
    g = torch.ones_like(u)
    p.lens_vjp(0, lens, u, g)
    t0 = time.perf_counter()
    for _ in range(reps):
        p.lens_vjp(0, lens, u, g)
    t_vjp = (time.perf_counter() - t0) / reps
    out = {"grid": inst.n, "threshold_of_peak": 0.01, "hot_areas": count,
           "hot_areas_us": t_hot * 1e6, "moment_us": t_mom * 1e6, "lens_us": t_lens * 1e6,
           "lens_vjp_us": t_vjp * 1e6}
    if not args.no_cpu:
        from oracle import diagnostics as D
        wh = w.cpu().numpy()
        t0 = time.perf_counter()
        want = D.hot_area_count(wh, thr)
        out["cpu_oracle_hot_areas_us"] = (time.perf_counter() - t0) * 1e6
        out["matches_oracle"] = bool(want == count)
    return out


def run_ga(args):
    """One generation of the genetic search: 8 theta vectors of the 256^2
    single-filament beam marched 500 steps as one batch, fitness read back."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.ga import population_evaluator
    from paper_2306_15678_amd.march import Propagator, desc_of
    inst = W.config4_sparse()
    pop_n = 8
    rng = np.random.default_rng(0)
    pop = [np.array(inst.theta) + 0.05 * rng.standard_normal(8) for _ in range(pop_n)]
    p = Propagator([desc_of(inst)] * pop_n, precision=32)
    ev = population_evaluator(p, W.initial_field(inst), W.synthetic_target(inst, 44), inst.n_steps)
    ev(pop)
    reps = max(2, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ev(pop)
    t = (time.perf_counter() - t0) / reps
    p.close()
    gp = float(inst.n) ** 2 * inst.n_steps * pop_n
    return {"workload": f"{pop_n} theta vectors of the 256x256 single-filament beam, Kerr+ansatz, "
                        f"{inst.n_steps} z steps each, one batched march + fitness read-back",
            "ms_per_generation": t * 1e3, "value": gp / t, "unit": UNIT}


def parity_vs_stored(inst, power, peak, fluence):
    """The 1024^2 march against the oracle's stored samples of it (written
    by tests/golden/calibrate_floor.py c2); None if the fixture is absent."""
    path = os.path.join(ROOT, "tests", "golden", "floor_c2.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    ref = d["reference"]
    last = str(d["steps"][-1])
    bf = np.array(ref["block_fluence"][last])
    b = inst.n // bf.shape[0]
    got = fluence.reshape(bf.shape[0], b, bf.shape[0], b).mean(axis=(1, 3))
    k = d["steps"].index(int(last))
    return {
        "z_steps": int(last),
        "block_fluence_rel_l2": float(np.linalg.norm(got - bf) / np.linalg.norm(bf)),
        "power_max_rel_err": float(np.max(np.abs(np.array(power) / np.array(ref["power"]) - 1))),
        "peak_final_rel_err": float(abs(peak[-1] / ref["peak"][-1] - 1)),
        "floor_peer32_block_fluence": d["peer32"]["block_fluence"][k],
    }


def measured_copy_peak(gib=4):
    """HBM bandwidth by a STREAM-style copy: a 4 GiB buffer into another
    (read + write counted), median of 5, torch events on torch's stream."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    t = sorted(ts)[len(ts) // 2]
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * gib * (1 << 30) / t / 1e9


def cpu_baseline(steps=1):
    """The FP64 oracle (numpy) on a bounded sample of the headline workload:
    forward + adjoint of its first `steps` z steps on the full 4096^2 grid,
    single-threaded, and again with the oracle's 2-D FFTs through scipy.fft
    on the host's cores."""
    import workloads as W
    from oracle import march as M

    inst = W.config5()[0]
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 5)
    pts = float(inst.n) ** 2 * steps

    def run():
        t0 = time.perf_counter()
        M.gradient(u0, inst, n_steps=steps, cotangent=lambda u: M.fluence_loss(u, target))
        return time.perf_counter() - t0

    dt = run()
    host = os.cpu_count() or 1
    workers = min(host, 16)
    with M.fft_workers(workers):
        dtw = run()
    return {
        "value": pts / dt,
        "unit": UNIT,
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 numpy oracle, forward + adjoint of the first {steps} z steps of the "
                  f"4096x4096 headline march ({dt:.1f} s, single-threaded numpy FFT)",
        "host_cpu_count": host,
        "threaded": {"value": pts / dtw, "unit": UNIT, "cores": workers,
                     "sample": f"the same with the oracle's 2-D FFTs through scipy.fft, "
                               f"workers={workers} ({dtw:.1f} s)"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="checkpoint interval of the recorded march (0: keep the whole "
                         "trajectory when it fits half the free HBM, else about sqrt(steps))")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only (no 1024^2, batch, GA or scheme legs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (a beam or a batch of beams marches on one "
              "device; there is no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    inst = W.config5()[0]
    head = run_headline(args)
    copy_peak = measured_copy_peak()
    t32 = head["fp32"]["s_per_step"]
    m = head["fp32"]["ckpt_every"]
    k = head["fp32"]["stored_segments"]
    rec = head["fp32"]["recomputed_steps"]
    # whole-march algorithmic bytes per grid point and z step (complex64):
    # forward 32, adjoint 40 (its row pass reads the stored V), and 32 per
    # recomputed step; recording writes nothing beyond the march's own output
    design_bytes = 72.0 + 32.0 * rec / inst.n_steps
    march_gbps = head["fp32"]["value"] * design_bytes / 1e9
    # the same march priced per step as stored (80 B) or recomputed (112 + 8/M B)
    f_rec = rec / inst.n_steps
    survey_bytes = 80.0 * (1.0 - f_rec) + (112.0 + 8.0 / m) * f_rec
    line = {
        "metric": METRIC,
        "value": head["fp32"]["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "large-aperture beam, 4096x4096 complex64 (FP64 reductions), "
                        "Kerr+MPA+plasma+ansatz, 50 Kolmogorov screens over 1 km, 5000 z steps, "
                        f"forward+adjoint, checkpoint every {m} steps, last {k} segments "
                        f"kept whole ({rec} steps recomputed)",
            "grid": inst.n, "z_steps": inst.n_steps, "ckpt_every": m,
            "stored_segments": k, "recomputed_steps": rec,
            "workspace_GiB": round(head["fp32"]["workspace_GiB"], 2),
            "beam": "w0=2.5 cm, 1000 P_cr, 5% seeded noise, window 12 cm, dz=20 cm",
        },
        "roofline": roofline(head, copy_peak),
        "march_hbm": {
            "bytes_per_gp_step": design_bytes,
            "achieved_GBps": march_gbps,
            "frac": march_gbps / HBM_PEAK_GBS,
            "note": "whole-march algorithmic bytes (forward 32, adjoint 40, 32 per recomputed "
                    "step, per grid point and z step) x grid-point.steps/s over the 8 TB/s spec",
            "survey_basis": {
                "bytes_per_gp_step": survey_bytes,
                "achieved_GBps": head["fp32"]["value"] * survey_bytes / 1e9,
                "frac": head["fp32"]["value"] * survey_bytes / 1e9 / HBM_PEAK_GBS,
                "note": "the same throughput on 80 B per grid-point step where the pre-screen "
                        "field is stored (forward 32 + 8 to store it, adjoint 40) and "
                        "112 + 8/M B where it is recomputed from checkpoints every M steps, "
                        "weighted by the recomputed fraction of the march",
            },
        },
        "passes_ms": head["passes"],
        "forward_only": {"value": head["fwd"]["value"],
                         "ms_per_march": head["fwd"]["s_per_step"] * 1e3},
        "tile_variants_fp32": head["fp32"]["tune"],
        "power_end_over_start": head["power_end_over_start"],
    }
    if "fp64" in head:
        line["fp64"] = {"value": head["fp64"]["value"], "ms_per_step": head["fp64"]["s_per_step"] * 1e3,
                        "ckpt_every": head["fp64"]["ckpt_every"],
                        "stored_segments": head["fp64"]["stored_segments"],
                        "speedup_fp32_over_fp64": head["fp64"]["s_per_step"] / t32}
        line["fp32_vs_fp64"] = head["fp32_vs_fp64"]
    if not args.no_extra:
        _say("1024^2 forward+adjoint")
        line["multifilament_fwd_adj"] = run_c2_fwd_adj(args)
        _say("64-beam batch")
        line["batched_forward"], line["batched_fwd_adj"] = run_batched(args)
        _say("GA generation, schemes")
        line["ga_generation"] = run_ga(args)
        line.update(run_schemes(args))
    if not args.no_cpu:
        _say("CPU oracle")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
