"""Rounding floors of the split-step march, computed with the FP64 oracle only.

Filamentation is chaotic: modulational instability and collapse amplify any
perturbation, so two correct discretisations that differ only in rounding
drift apart.  The tolerance of a GPU run against the FP64 oracle is
therefore stated relative to a floor measured on the oracle itself:

* ``in64`` / ``in32``: rel L2 between the oracle run from U0 and from
  U0 (1 + eps eta) with eps = 2^-53 / 2^-24 and eta a unit complex normal
  (a one-time perturbation at the input);
* ``step32`` / ``step64``: the same, but a perturbation of size
  eps sqrt(4 log2 N + 4) injected at every step (the expected relative
  rounding of one FP32/FP64 step: four length-N FFTs plus pointwise
  multiplies), maximum over two noise seeds;
* ``peer32``: rel L2 between the oracle and an independent complex64
  implementation of the same discrete map (torch on the CPU, normalised
  intensity x = I/I_a, FP32 tables, FFTs and screen).  FP32 rounding of
  tables, twiddles and coefficients acts coherently from step to step, which
  the random models above do not capture; this peer measures it directly.
* ``peer64``: the same independent implementation in complex128 (torch
  CPU), for the coherent FP64 table rounding.

Writes tests/golden/floor_<name>.json with the field and fluence floors at
the listed step counts, and the oracle's own samples of the reference run at
the same steps (total power and peak intensity after every step, the
fluence averaged over 32x32 blocks at a quarter, half, three quarters and
all of the march, and the field at 64 seeded grid points), which full-size GPU tests compare against.  Usage:
    python tests/golden/calibrate_floor.py c1
    python tests/golden/calibrate_floor.py c2 --steps 2000 --every 100
"""
import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import march as M  # noqa: E402


def _eta(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def floors(inst, n_steps, every, screens=None):
    u0 = W.initial_field(inst)
    marks = list(range(every, n_steps + 1, every))
    # reference trajectory
    ref = {}
    power, peak = [], []
    u = u0.copy()
    done = 0
    for m in marks:
        r = M.march(u, inst, n_steps=m - done, screens=_shift(screens, done))
        u = r.field
        power += r.power.tolist()
        peak += r.peak.tolist()
        done = m
        ref[m] = u
    out = {"steps": marks}
    pts = np.random.default_rng(777).integers(0, inst.n, size=(64, 2))
    out["sample_points"] = pts.tolist()
    out["reference"] = {
        "power": power, "peak": peak,
        "block_fluence": {str(m): M.block_mean(np.abs(ref[m]) ** 2, inst.n // 32).tolist()
                          for m in _quarters(marks)},
        "field_re": {str(m): ref[m][pts[:, 0], pts[:, 1]].real.tolist() for m in marks},
        "field_im": {str(m): ref[m][pts[:, 0], pts[:, 1]].imag.tolist() for m in marks},
    }
    rng = np.random.default_rng(12345)
    for name, eps in (("in64", 2.0 ** -53), ("in32", 2.0 ** -24)):
        u = u0 * (1 + eps * _eta(rng, u0.shape))
        done = 0
        f, w = [], []
        for m in marks:
            u = M.march(u, inst, n_steps=m - done, screens=_shift(screens, done)).field
            done = m
            f.append(M.rel_l2(u, ref[m]))
            w.append(M.rel_l2(np.abs(u) ** 2, np.abs(ref[m]) ** 2))
        out[name] = {"field": f, "fluence": w}
    amp = math.sqrt(4 * math.log2(inst.n) + 4)
    for name, eps in (("step64", 2.0 ** -53 * amp), ("step32", 2.0 ** -24 * amp)):
        fmax = np.zeros(len(marks))
        wmax = np.zeros(len(marks))
        for seed in (1, 2):
            r = np.random.default_rng(seed)
            u = u0.copy()
            k = 0
            for n in range(n_steps):
                u = u * (1 + eps * _eta(r, u.shape))
                u = M.march(u, inst, n_steps=1, screens=_shift(screens, n)).field
                if n + 1 == marks[k]:
                    fmax[k] = max(fmax[k], M.rel_l2(u, ref[marks[k]]))
                    wmax[k] = max(wmax[k], M.rel_l2(np.abs(u) ** 2, np.abs(ref[marks[k]]) ** 2))
                    k += 1
        out[name] = {"field": fmax.tolist(), "fluence": wmax.tolist()}
    out["peer32"] = peer_floors(inst, marks, screens, ref, power, peak)
    return out


def peer_floors(inst, marks, screens, ref, power, peak, bits=32):
    """Field, fluence, block-fluence and diagnostic floors of the complex64
    (bits=32) or complex128 (bits=64) peer against the oracle reference."""
    peer = peer32(inst, marks, screens, bits)
    pp = np.array(peer["diag"]["power"])
    pk = np.array(peer["diag"]["peak"])
    b = max(1, inst.n // 32)
    return {
        "field": [M.rel_l2(peer[m], ref[m]) for m in marks],
        "fluence": [M.rel_l2(np.abs(peer[m]) ** 2, np.abs(ref[m]) ** 2) for m in marks],
        "block_fluence": [M.rel_l2(M.block_mean(np.abs(peer[m]) ** 2, b),
                                   M.block_mean(np.abs(ref[m]) ** 2, b)) for m in marks],
        # largest relative difference of power / peak over steps 1..m
        "power": [float(np.max(np.abs(pp[:m] / np.array(power[:m]) - 1))) for m in marks],
        "peak": [float(np.max(np.abs(pk[:m] / np.array(peak[:m]) - 1))) for m in marks],
    }


def _quarters(marks):
    """The marks nearest to 1/4, 1/2, 3/4 and all of the march."""
    last = marks[-1]
    out = []
    for q in (0.25, 0.5, 0.75, 1.0):
        m = min(marks, key=lambda v: abs(v - q * last))
        if m not in out:
            out.append(m)
    return out


def peer32(inst, marks, screens=None, bits=32):
    """complex64 (bits=64: complex128) march of the same map (torch CPU),
    normalised units."""
    import torch
    cdt, rdt = (np.complex64, np.float32) if bits == 32 else (np.complex128, np.float64)
    tdt = torch.float32 if bits == 32 else torch.float64
    m = inst.medium
    th = [float(v) for v in (inst.theta or (0.0,) * 8)]
    n = inst.n
    k0 = 2.0 * math.pi / m.wavelength
    k = 2.0 * math.pi * np.fft.fftfreq(n, d=inst.length / n)
    prop = np.exp(-1j * (k[None, :] ** 2 + k[:, None] ** 2) * inst.dz / (2 * k0))
    P = torch.from_numpy(prop.astype(cdt))
    cK = torch.tensor(k0 * m.n2 * m.i_ref * inst.dz, dtype=tdt)
    K = m.mpa_order
    cM = torch.tensor((K - 1) * m.beta_k * m.i_ref ** (K - 1) * inst.dz, dtype=tdt)
    u = torch.from_numpy((W.initial_field(inst) / math.sqrt(m.i_ref)).astype(cdt))
    out = {}
    diag = {"power": [], "peak": []}
    dx2 = (inst.length / n) ** 2
    for step in range(1, marks[-1] + 1):
        v = torch.fft.ifft2(P * torch.fft.fft2(u))
        x = (v.real ** 2 + v.imag ** 2)
        ph = torch.zeros_like(x)
        la = torch.zeros_like(x)
        if m.terms & W.TERM_KERR:
            ph = ph + cK * x
        if m.terms & W.TERM_PLASMA:
            ph = ph - cK * x ** K / (1 + x ** (K - 1))
        if m.terms & W.TERM_MPA:
            la = la - torch.log(1 + cM * x ** (K - 1)) / (2 * (K - 1))
        if m.terms & W.TERM_ANSATZ:
            den = 1 + x ** 4
            ph = ph + cK * sum(th[q - 1] * x ** q for q in range(1, 5)) / den
            la = la - cK * sum(th[3 + q] * x ** q for q in range(1, 5)) / den
        if screens and (step - 1) in screens:
            ph = ph + torch.from_numpy(screens[step - 1].astype(rdt))
        u = v * torch.exp(la) * torch.polar(torch.ones_like(ph), ph)
        inten = (u.real.double() ** 2 + u.imag.double() ** 2) * m.i_ref
        diag["power"].append(float(inten.sum()) * dx2)
        diag["peak"].append(float(inten.max()))
        if step in marks:
            out[step] = u.numpy().astype(np.complex128) * math.sqrt(m.i_ref)
    out["diag"] = diag
    return out


def peer32_loss(inst, steps, target):
    """complex64 peer of march + fluence loss (torch CPU) with its gradient
    by reverse autodiff: (loss, dL/dU0 [SI], dL/dtheta)."""
    import torch
    m = inst.medium
    n = inst.n
    k0 = 2.0 * math.pi / m.wavelength
    k = 2.0 * math.pi * np.fft.fftfreq(n, d=inst.length / n)
    prop = np.exp(-1j * (k[None, :] ** 2 + k[:, None] ** 2) * inst.dz / (2 * k0))
    P = torch.from_numpy(prop.astype(np.complex64))
    cK = float(k0 * m.n2 * m.i_ref * inst.dz)
    K = m.mpa_order
    cM = float((K - 1) * m.beta_k * m.i_ref ** (K - 1) * inst.dz)
    sa = math.sqrt(m.i_ref)
    u0 = torch.from_numpy((W.initial_field(inst) / sa).astype(np.complex64)).requires_grad_(True)
    th = torch.tensor([float(v) for v in (inst.theta or (0.0,) * 8)], dtype=torch.float32,
                      requires_grad=True)
    u = u0
    for _ in range(steps):
        v = torch.fft.ifft2(P * torch.fft.fft2(u))
        x = v.real ** 2 + v.imag ** 2
        ph = torch.zeros_like(x)
        la = torch.zeros_like(x)
        if m.terms & W.TERM_KERR:
            ph = ph + cK * x
        if m.terms & W.TERM_PLASMA:
            ph = ph - cK * x ** K / (1 + x ** (K - 1))
        if m.terms & W.TERM_MPA:
            la = la - torch.log(1 + cM * x ** (K - 1)) / (2 * (K - 1))
        if m.terms & W.TERM_ANSATZ:
            den = 1 + x ** 4
            ph = ph + cK * sum(th[q - 1] * x ** q for q in range(1, 5)) / den
            la = la - cK * sum(th[3 + q] * x ** q for q in range(1, 5)) / den
        u = v * torch.exp(la) * torch.polar(torch.ones_like(ph), ph)
    tg = torch.from_numpy((target / m.i_ref).astype(np.float32))
    inten = u.real ** 2 + u.imag ** 2
    loss = ((inten - tg) ** 2).sum() / (tg ** 2).sum()
    loss.backward()
    return (float(loss), u0.grad.numpy().astype(np.complex128) / sa,
            th.grad.numpy().astype(np.float64))


def gradient_floors(inst, marks, target):
    """Floors of (loss, dL/dU0, dL/dtheta) against the FP64 oracle: the
    oracle itself from an input perturbed by 2^-53 and the complex64 peer."""
    u0 = W.initial_field(inst)
    rng = np.random.default_rng(54321)
    pert = u0 * (1 + 2.0 ** -53 * _eta(rng, u0.shape))
    out = {"steps": marks, "in64": [], "peer32": []}

    def cot(u):
        return M.fluence_loss(u, target)
    for m in marks:
        l0, g0, t0 = M.gradient(u0, inst, n_steps=m, cotangent=cot)
        l1, g1, t1 = M.gradient(pert, inst, n_steps=m, cotangent=cot)
        l2, g2, t2 = peer32_loss(inst, m, target)
        tn = np.max(np.abs(t0))
        out["in64"].append([abs(l1 / l0 - 1), M.rel_l2(g1, g0), float(np.max(np.abs(t1 - t0)) / tn)])
        out["peer32"].append([abs(l2 / l0 - 1), M.rel_l2(g2, g0), float(np.max(np.abs(t2 - t0)) / tn)])
    return out


def _shift(screens, offset):
    if not screens:
        return None
    return {k - offset: v for k, v in screens.items() if k - offset >= 0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", help="c1, c2, c3:<beam> or c4")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--peer-only", action="store_true",
                    help="recompute only the complex64-peer floors into the existing file")
    ap.add_argument("--peer-bits", type=int, default=32, choices=(32, 64),
                    help="with --peer-only: the complex64 (32) or complex128 (64) peer")
    ap.add_argument("--floors-only", action="store_true",
                    help="omit the reference samples (the test runs the oracle itself)")
    args = ap.parse_args()
    screens = None
    if args.config.startswith("c3:"):
        from oracle import turbulence as T
        inst = W.config3()[int(args.config[3:])]
        screens = T.instance_screens(inst)
    else:
        inst = {"c1": W.config1, "c2": W.config2, "c4": W.config4,
                "c5": W.config5}[args.config]()[0]
    n_steps = args.steps or inst.n_steps
    path = os.path.join(HERE, "floor_%s.json" % args.config.replace(":", "_"))
    if args.peer_only:
        res = json.load(open(path))
        marks = res["steps"]
        u = W.initial_field(inst)
        ref, power, peak, done = {}, [], [], 0
        for m in marks:
            r = M.march(u, inst, n_steps=m - done, screens=_shift(screens, done))
            u = r.field
            power += r.power.tolist()
            peak += r.peak.tolist()
            done = m
            ref[m] = u
        name = "peer%d" % args.peer_bits
        res[name] = peer_floors(inst, marks, screens, ref, power, peak, args.peer_bits)
        with open(path, "w") as f:
            json.dump(res, f, indent=1)
        for k, v in res[name].items():
            print(name, k, ["%.1e" % x for x in v])
        return
    res = floors(inst, n_steps, args.every, screens)
    if args.config == "c4":
        res["gradient"] = gradient_floors(inst, [100, res["steps"][-1]],
                                          W.synthetic_target(inst, 44))
        for k in ("in64", "peer32"):
            print("gradient", k, [["%.1e" % v for v in row] for row in res["gradient"][k]])
    if args.floors_only:
        res.pop("reference")
        res.pop("sample_points")
    res["config"] = args.config
    res["n"] = inst.n
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    for k in ("in64", "in32", "step64", "step32", "peer32"):
        print(k, "field", ["%.1e" % x for x in res[k]["field"]])
        print(k, "fluence", ["%.1e" % x for x in res[k]["fluence"]])


if __name__ == "__main__":
    main()
