"""Throughput of the split-step march on one MI355X (grid-point . steps / s).

Workload (default): the 1024 x 1024 multifilamentation beam (1 cm, 100 P_cr,
Kerr + multiphoton absorption + saturating plasma, 10 % seeded noise),
2000 z steps of 1 cm, complex64 with FP64 reductions.  One bench step is
the whole differentiable march: the recorded forward march (the whole
trajectory kept in HBM when it fits half the free memory, 16 GiB here;
otherwise checkpoints with segment recompute in the backward), the
fluence-mismatch loss against a synthetic target, and the exact adjoint
back to the input field.  Grid-point . steps
count each z step once.

The JSON line also carries: the roofline of the dominant pass kernel
(HIP events around that pass at every 100th step of the timed marches,
recorded on the library's stream inside its step graphs), the
same march with the complex128 instantiation of the kernels, forward-only
throughput, parity against the oracle's stored samples of this workload,
and the FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SAMPLE_EVERY = 100
METRIC = "grid-point·steps/s SSFM fwd+adjoint, FP32 vs FP64, at stated L2 error"


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


def run_gpu(args):
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator

    torch.cuda.set_device(0)
    inst = W.config2()[0]
    n, z_steps = inst.n, inst.n_steps
    ckpt = args.ckpt_every
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 2)
    dev = torch.device("cuda", 0)
    u0_d = torch.from_numpy(u0).to(dev)
    tgt_d = torch.from_numpy(target).to(dev)
    gp_steps = float(n) * n * z_steps
    out = {}

    def make(precision):
        from paper_2306_15678_amd.march import checkpoint_interval
        from paper_2306_15678_amd.tune import tune
        m = ckpt or checkpoint_interval(_desc_list([inst]), precision, z_steps)
        out["ckpt_fp%d" % precision] = m
        p = Propagator(_desc_list([inst]), precision=precision, max_steps=z_steps,
                       ckpt_every=m, device=dev)
        if precision == 32 and args.variants:
            # tile variants given on the command line (a profiled run pins the
            # ones an unprofiled run chose: the profiler perturbs the tuner)
            r, c = (int(v) for v in args.variants.split(","))
            p.select_plan(inst.n, r, c)
            out["tune_fp32"] = {"row": r, "col": c, "pinned": True}
        else:
            # pick the fastest tile variants (setup, not timed)
            out["tune_fp%d" % precision] = tune(p, reps=30, use_cache=False)[inst.n]
        return p

    def fwd_adj(p):
        p.set_field(0, u0_d)
        p.forward_record(z_steps)
        p.fluence_loss(0, tgt_d)
        p.backward()

    for precision in (32, 64):
        p = make(precision)
        if precision == 32:
            # HIP events around the row and column pass of every 100th step of
            # each forward march, inside the captured step graphs
            p.set_pass_timing(SAMPLE_EVERY)
        t = _timed(lambda: fwd_adj(p), args.steps if precision == 32 else max(1, args.steps // 2),
                   args.warmup, p.synchronize)
        out[precision] = {"s_per_step": t, "value": gp_steps / t}
        if precision == 32:
            # pass durations sampled in the forward record of the last timed step
            ms_row, ms_col, n_samp = p.pass_times()
            out["live"] = {"ms_row": ms_row, "ms_col": ms_col, "samples": n_samp}
            # forward only (plain propagate) on the same context
            def fwd():
                p.set_field(0, u0_d)
                p.propagate(z_steps)
            tf = _timed(fwd, args.steps, 1, p.synchronize)
            out["fwd"] = {"s_per_step": tf, "value": gp_steps / tf}
            # parity of the timed march: loss, diagnostics and fluence
            p.set_field(0, u0_d)
            p.propagate(z_steps)
            pw, pk = p.diag(0, z_steps)
            fl = p.intensity(0)
            out["parity"] = parity_vs_stored(inst, pw, pk, fl, p.field(0))
            out["diagnostics"] = time_diagnostics(p, inst, args)
            # each pass alone, 200 back-to-back launches (the tuner's timing)
            ms_row, ms_col, b_row, b_col = p.time_passes(reps=200)
            out["passes"] = {"ms_row": ms_row, "ms_col": ms_col,
                             "bytes_row": b_row, "bytes_col": b_col}
        p.close()
        del p
        torch.cuda.empty_cache()
    return out


def run_batched(args):
    """Forward march of the 64 uneven beams with turbulence screens
    (n in {256, 512, 768, 1024}, 2000 steps), one context, graph-captured."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator
    from paper_2306_15678_amd.tune import tune

    insts = W.config3()
    p = Propagator(_desc_list(insts), precision=32, device=torch.device("cuda", 0))
    tune(p, reps=10, use_cache=False)
    p.gen_screens()
    fields = [torch.from_numpy(W.initial_field(i)).to("cuda") for i in insts]

    def fwd():
        for b, u in enumerate(fields):
            p.set_field(b, u)
        p.propagate(insts[0].n_steps)

    # every 40th step: the beams' screens act after steps 49, 149, ..., which
    # every 100th step (50, 150, ...) would always hit; these samples are
    # the typical, screen-free step
    p.set_pass_timing(40)
    t = _timed(fwd, max(1, args.steps // 5), 1, p.synchronize)
    ms_row, ms_col, n_samp = p.pass_times()
    _, _, b_row, _ = p.time_passes(reps=1)
    gp = float(sum(i.n * i.n for i in insts)) * insts[0].n_steps
    p.close()
    return {"s_per_step": t, "value": gp / t, "ms_row": ms_row, "ms_col": ms_col,
            "samples": n_samp, "bytes_pass": b_row}


FD_ITERS = 4


def run_schemes(args):
    """The scheme variants on the 1024^2 workload, complex64, forward march:
    Strang splitting (2000 steps) beside Lie; the finite-difference reference
    scheme (500 steps, FD_ITERS iterations per step) with its whole-step HBM
    rate; and the cost of 3 subharmonic levels in the screen synthesis of
    the 64-beam batch."""
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
    out["strang_forward"] = {"z_steps": inst.n_steps, "value": gp / t_strang,
                             "unit": "grid-point\u00b7steps/s", "ms_per_march": t_strang * 1e3,
                             "lie_ms_per_march": t_lie * 1e3}
    fd_steps = 500
    p.set_finite_difference(FD_ITERS)
    t_fd = _timed(fwd(fd_steps), reps, 1, p.synchronize)
    pw, _ = p.diag(0, fd_steps)
    field_bytes = 8.0 * n * n
    # per step: FD_ITERS column passes (Wk read + written), FD_ITERS - 1 row
    # passes (Wk and S read, Wk written), the finishing row pass (Wk and S
    # read, S and Wk written)
    step_bytes = field_bytes * (2 * FD_ITERS + 3 * (FD_ITERS - 1) + 4)
    us_step = t_fd / fd_steps * 1e6
    out["fd_reference"] = {
        "workload": f"{n}x{n} complex64, Kerr+MPA+plasma, {fd_steps} z steps, "
                    f"{FD_ITERS} fixed-point iterations per step",
        "value": float(n) * n * fd_steps / t_fd, "unit": "grid-point\u00b7steps/s",
        "us_per_step": us_step, "launches_per_step": 2 * FD_ITERS,
        "bytes_per_step": step_bytes, "achieved_GBps": step_bytes / (us_step * 1e-6) / 1e9,
        "frac_of_8TBps": step_bytes / (us_step * 1e-6) / 8e12,
        "power_drift": float(abs(pw[-1] / pw[0] - 1))}
    p.close()
    del p
    torch.cuda.empty_cache()
    insts = W.config3()
    q = Propagator(_desc_list(insts), precision=32, device=dev)
    t0 = _timed(q.gen_screens, 5, 1, q.synchronize)
    for b in range(len(insts)):
        q.set_subharmonics(b, 3)
    t3 = _timed(q.gen_screens, 5, 1, q.synchronize)
    q.close()
    pts = float(sum(i.n * i.n * i.n_screens for i in insts))
    out["subharmonics"] = {"workload": "64 beams x 20 screens, n in 256..1024, 3 levels",
                           "gen_screens_ms": t0 * 1e3, "with_3_levels_ms": t3 * 1e3,
                           "ns_per_screen_point": (t3 - t0) / pts * 1e9}
    return out


def run_large(args, copy_peak):
    """Forward march of the 4096^2 large-aperture beam (Kerr, MPA, plasma,
    ansatz, 50 turbulence screens), the first 500 of its 5000 steps,
    complex64, passes sampled in-march as for the headline: the same kernels
    with four wavefronts per SIMD."""
    import torch

    import workloads as W
    from paper_2306_15678_amd.march import Propagator
    from paper_2306_15678_amd.tune import tune

    dev = torch.device("cuda", 0)
    inst = W.config5()[0]
    n, steps = inst.n, 500
    p = Propagator(_desc_list([inst]), precision=32, device=dev)
    tune(p, reps=10, use_cache=False)
    p.gen_screens()
    p.set_theta(0, inst.theta)
    u0_d = torch.from_numpy(W.initial_field(inst)).to(dev)

    def fwd():
        p.set_field(0, u0_d)
        p.propagate(steps)

    # every 40th step (steps 20, 60, ...): screens act after steps 49, 149,
    # ..., which sampling every 100th step (steps 50, 150, ...) would hit
    # each time; these samples are the typical, screen-free step
    p.set_pass_timing(40)
    t = _timed(fwd, max(1, args.steps // 5), 1, p.synchronize)
    ms_row, ms_col, n_samp = p.pass_times()
    p.close()
    torch.cuda.empty_cache()
    dom = max(ms_row, ms_col)
    gbps = 16.0 * n * n / (dom * 1e-3) / 1e9
    return {"workload": f"{n}x{n} complex64, Kerr+MPA+plasma+ansatz, 50 Kolmogorov screens, "
                        f"first {steps} of 5000 z steps, forward",
            "value": float(n) * n * steps / t, "unit": "grid-point\u00b7steps/s",
            "ms_per_march": t * 1e3, "passes_ms": {"row": ms_row, "col": ms_col},
            "samples": n_samp, "timing": "HIP events around the passes of every 40th step "
                                          "(screen-free steps), library stream",
            "dominant_pass_GBps": gbps,
            "dominant_pass_frac": gbps / HBM_PEAK_GBS,
            "dominant_pass_frac_of_measured_copy": gbps / copy_peak}


def time_diagnostics(p, inst, args):
    """The paper's beam diagnostics on the end fluence of the march: hot-area
    count (4-connected regions above 1 % of the peak, periodic window), the
    energy moment Q(1, 1) and one effective-lens screen, per call including
    the host synchronisation; the oracle's count on the same FP64 array
    beside it."""
    w = p.intensity(0, device=True)
    thr = 0.01 * float(w.max())
    reps = max(5, args.steps)
    count = p.hot_areas(w, thr)
    t0 = time.perf_counter()
    for _ in range(reps):
        p.hot_areas(w, thr)
    t_hot = (time.perf_counter() - t0) / reps
    p.moment(w, inst.length, 1.0, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        p.moment(w, inst.length, 1.0, 1)
    t_mom = (time.perf_counter() - t0) / reps
    # effective-lens screen (filter through the pass kernels + pointwise
    # lens), scaled to this fluence; it changes the field, so it runs last
    from paper_2306_15678_amd.march import make_lens
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
    # its vector-Jacobian product (input cotangent and parameter gradients)
    import torch
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


def measured_copy_peak(gib=4):
    """HBM bandwidth of this device by a STREAM-style copy: one 4 GiB buffer
    into another (read + write counted), median of 5, timed with torch
    events on torch's current stream (where the copy runs)."""
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


def traffic_per_launch(kind, variant):
    """HBM bytes per launch of the forward ``kind`` pass ("row" or "col") of
    tile ``variant`` on the 1024^2 grid, from the committed FETCH_SIZE and
    WRITE_SIZE summary, each counter scaled by its own reading for a plain
    copy kernel of known size.  None when the summary is absent or was taken
    on other kernel sources."""
    from paper_2306_15678_amd.passprof import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "traffic_c2_1024.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    c = d["copy_kernel"]
    for e in d.get(kind, []):
        if e["variant"] == variant:
            return 1024.0 * (e["fetch_kib"] / c["fetch_scale"] + e["write_kib"] / c["write_scale"])
    return None


def run_ga(args):
    """One generation of the genetic search: 8 individuals (theta vectors)
    of the 256^2 single-filament beam marched 500 steps as one batch, and
    their fitness read back."""
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
    reps = max(2, args.steps // 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ev(pop)
    t = (time.perf_counter() - t0) / reps
    p.close()
    gp = float(inst.n) ** 2 * inst.n_steps * pop_n
    return {"workload": f"{pop_n} theta vectors of the 256x256 single-filament beam, Kerr+ansatz, "
                        f"{inst.n_steps} z steps each, one batched march + fitness read-back",
            "ms_per_generation": t * 1e3, "value": gp / t, "unit": "grid-point·steps/s"}


def parity_vs_stored(inst, power, peak, fluence, field):
    """Compare with the oracle's samples of this workload (written by
    tests/golden/calibrate_floor.py c2); None if the fixture is absent."""
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
        "floor_step32_fluence": d["step32"]["fluence"][k],
        "floor_step32_field": d["step32"]["field"][k],
    }


def cpu_baseline(seconds_target=15.0):
    """The FP64 oracle (numpy) on a bounded sample: forward + adjoint of the
    first z steps of the same 1024^2 beam."""
    import workloads as W
    from oracle import march as M

    inst = W.config2()[0]
    u0 = W.initial_field(inst)
    target = W.synthetic_target(inst, 2)
    steps = 4
    t0 = time.perf_counter()
    M.gradient(u0, inst, n_steps=steps, cotangent=lambda u: M.fluence_loss(u, target))
    dt = time.perf_counter() - t0
    steps = max(steps, int(steps * seconds_target / max(dt, 1e-3)))
    steps = min(steps, 200)
    t0 = time.perf_counter()
    M.gradient(u0, inst, n_steps=steps, cotangent=lambda u: M.fluence_loss(u, target))
    dt = time.perf_counter() - t0
    return {
        "value": float(inst.n) ** 2 * steps / dt,
        "unit": "grid-point·steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"FP64 numpy oracle, forward + adjoint of the first {steps} z steps of the "
                  f"1024x1024 workload ({dt:.1f} s, single-threaded pocketfft)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="checkpoint interval of the recorded march (0: keep the whole "
                         "trajectory when it fits half the free HBM, else about sqrt(steps))")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--variants", default="",
                    help="ROW,COL: tile variants of the 1024^2 complex64 passes instead of "
                         "tuning them (FP32 march only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the march of one beam or a batch lives "
              "on one device; there is no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    inst = W.config2()[0]
    g = run_gpu(args)
    copy_peak = measured_copy_peak()
    t32, t64 = g[32]["s_per_step"], g[64]["s_per_step"]
    ps, lv = g["passes"], g["live"]
    dom = "col" if lv["ms_col"] >= lv["ms_row"] else "row"
    ms = lv["ms_" + dom]
    achieved = ps["bytes_" + dom] / (ms * 1e-3) / 1e9
    traffic = traffic_per_launch(dom, g["tune_fp32"][dom])
    line = {
        "metric": METRIC,
        "value": g[32]["value"],
        "unit": "grid-point·steps/s",
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
            "workload": "multifilamentation beam, 1024x1024 complex64 (FP64 reductions), "
                        "Kerr+MPA+plasma, 2000 z steps, forward+adjoint, checkpoint every "
                        f"{g['ckpt_fp32']} steps",
            "grid": inst.n, "z_steps": inst.n_steps, "ckpt_every": g["ckpt_fp32"],
            "beam": "w0=1 cm, 100 P_cr, 10% seeded noise, window 6 cm, dz=1 cm",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom} pass (forward, complex64)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "measured_copy_GBps": copy_peak,
            "frac_of_measured_copy": achieved / copy_peak,
            "traffic": traffic,
            "traffic_over_algorithmic": (traffic / ps["bytes_" + dom]) if traffic else None,
            "ms_per_launch": ms,
            "bytes_per_launch": ps["bytes_" + dom],
            "timing": f"HIP events around the pass at every {SAMPLE_EVERY}th step of the "
                      f"forward record of the last timed step ({lv['samples']} samples), "
                      "library stream",
        },
        "fp64": {"value": g[64]["value"], "ms_per_step": t64 * 1e3, "ckpt_every": g["ckpt_fp64"],
                 "speedup_fp32_over_fp64": t64 / t32},
        "forward_only": {"value": g["fwd"]["value"], "ms_per_step": g["fwd"]["s_per_step"] * 1e3},
        "passes_ms": {"row": lv["ms_row"], "col": lv["ms_col"]},
        "isolated_passes_ms": {"row": ps["ms_row"], "col": ps["ms_col"]},
        "tile_variants": {"fp32": [g["tune_fp32"]["row"], g["tune_fp32"]["col"]],
                          "fp64": [g["tune_fp64"]["row"], g["tune_fp64"]["col"]]},
        "parity": g["parity"],
        "diagnostics": g["diagnostics"],
    }
    if not args.no_batched:
        bt = run_batched(args)
        dom_ms = max(bt["ms_row"], bt["ms_col"])  # sampled in the timed marches
        line["batched_forward"] = {
            "workload": "64 beams, n in {256,512,768,1024}, 20 Kolmogorov screens each, "
                        "Kerr+MPA+plasma, 2000 z steps, complex64, forward",
            "value": bt["value"], "unit": "grid-point·steps/s",
            "ms_per_march": bt["s_per_step"] * 1e3,
            "passes_ms": {"row": bt["ms_row"], "col": bt["ms_col"]},
            "timing": "HIP events around the passes of every 40th step (screen-free steps), "
                      "library stream",
            "dominant_pass_GBps": bt["bytes_pass"] / (dom_ms * 1e-3) / 1e9,
            "dominant_pass_frac": bt["bytes_pass"] / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "dominant_pass_frac_of_measured_copy":
                bt["bytes_pass"] / (dom_ms * 1e-3) / 1e9 / copy_peak,
        }
    if not args.no_batched:
        line["ga_generation"] = run_ga(args)
        line.update(run_schemes(args))
        line["large_grid"] = run_large(args, copy_peak)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
