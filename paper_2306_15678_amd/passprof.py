"""Short eager marches of every compiled tile variant, for hardware counters.

    python -m paper_2306_15678_amd.passprof [--precision 32] [--steps 4] [--large]
    python -m paper_2306_15678_amd.passprof --march ROW,COL,ROWADJ,COLADJ [--steps 4]
    python -m paper_2306_15678_amd.passprof --summarise FETCH.csv WRITE.csv --out T.json

On the 1024 x 1024 multifilamentation beam it selects each forward row-pass
variant in turn (column variant 0), then each column-pass variant (row
variant 0), and runs a recorded forward march of ``--steps`` steps with
graphs off, so that a counter profiler sees one plain dispatch per pass.
Each recorded march starts with one copy of the whole field into the first
checkpoint slot: a plain copy kernel of known size (n^2 complex elements
read and written) against which byte counters can be scaled.

Variants appear in index order: the k-th distinct forward row-pass kernel
name in dispatch order is row variant k, likewise for columns.  Last comes
an eager march of the finite-difference scheme (variant 0 plans).  With
``--large`` the beam is the 4096^2 large-aperture one (its Kerr, MPA and
plasma terms) and the finite-difference march is left out.  Prints one line
per phase; ``--out`` writes the layout as JSON.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys


# The sources the row and column pass kernels are compiled from.
PASS_SOURCES = ("fft_core.hpp", "plans.hpp", "screen.hpp", "internal.hpp", "kernels.hpp",
                "pass_kernels.hpp", "pass_row_f32.hip", "pass_row_f64.hip",
                "pass_col_f32.hip", "pass_col_f64.hip", "pass_col_hx.hpp",
                "pass_col_hx_f32.hip")


FD_ITERS = 4  # fixed-point iterations per finite-difference step


def kernel_source_hash() -> str:
    """SHA-256 over the pass kernels' sources: a byte counter taken on one
    hash describes the pass kernels of that hash only."""
    h = hashlib.sha256()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for name in PASS_SOURCES:
        h.update(name.encode())
        with open(os.path.join(here, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# pass kinds by kernel: (kernel template name, kind number) -> key
KIND_KEYS = {("k_row", 0): "row_fwd", ("k_col", 3): "col_fwd", ("k_col", 4): "col_adj",
             ("k_row", 1): "row_adj"}


def kernel_kind(name: str):
    """'row_fwd' / 'col_fwd' / 'col_adj' / 'row_adj' for a pass kernel's
    name (its last template argument is the pass kind), 'copy' for the
    calibration copy, None otherwise."""
    base = name.split("<")[0].split("::")[-1].strip()
    if base == "k_copy":
        return "copy"
    if base in ("k_row_pipe", "k_col_pipe"):  # persistent forms of the same passes
        base = base[:-len("_pipe")]
    if base == "k_col_hx":  # column passes exchanging through half the tile
        base = "k_col"
    if base in ("k_row", "k_col"):
        tail = name.rsplit(",", 1)[-1]
        digits = "".join(ch for ch in tail if ch.isdigit())
        if digits:
            return KIND_KEYS.get((base, int(digits)))
    return None


def _counter_rows(path: str):
    """(kernel name, counter, value, dispatch) rows of a rocprofv3 counter
    collection CSV (a file, or the directory holding one)."""
    import csv
    if os.path.isdir(path):
        found = [os.path.join(d, f) for d, _, fs in os.walk(path) for f in fs
                 if f.endswith("counter_collection.csv")]
        if not found:
            raise FileNotFoundError(f"no counter_collection.csv under {path}")
        path = found[0]
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            yield r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]), r["Dispatch_Id"]


def summarise(fetch: str, write: str, copy_bytes: float, out_json: str) -> dict:
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch, summed over the
    dispatch's counter instances) of each pass kind and of the calibration
    copy, with the copy's counter-per-byte scales; written as JSON for the
    bench's traffic figure."""
    per = {}
    for which, path in (("fetch", fetch), ("write", write)):
        acc = {}
        for name, counter, value, disp in _counter_rows(path):
            k = kernel_kind(name)
            if k is None:
                continue
            acc.setdefault(k, {}).setdefault(disp, [name, 0.0])[1] += value
        for k, d in acc.items():
            vals = [v for _, v in d.values()]
            e = per.setdefault(k, {"name": next(iter(d.values()))[0], "dispatches": len(vals)})
            e[which + "_kib"] = sum(vals) / len(vals)
    if "copy" not in per:
        raise RuntimeError("no calibration copy kernel among the dispatches")
    c = per.pop("copy")
    copy_kib = copy_bytes / 1024.0
    info = {"source_hash": kernel_source_hash(),
            "copy_kernel": {"name": c["name"], "bytes": copy_bytes,
                            "fetch_scale": c["fetch_kib"] / copy_kib,
                            "write_scale": c["write_kib"] / copy_kib},
            "kernels": per}
    with open(out_json, "w") as f:
        json.dump(info, f, indent=1)
    return info


def run_march(args) -> int:
    """The large-aperture 4096^2 beam with all its screen terms and
    turbulence: a recorded forward march of --steps steps, the fluence
    loss and the adjoint, graphs off, with the given tile variants, so that
    a counter profiler sees one plain dispatch per pass of every kind.  The
    record starts with one copy of the field (n^2 complex64 read and
    written), the calibration kernel."""
    import torch

    import workloads as W
    from .march import Propagator, desc_of
    inst = W.config5()[0]
    rv, cv, arv, acv = (int(x) for x in args.march.split(","))
    p = Propagator([desc_of(inst)], precision=32, max_steps=args.steps, ckpt_every=args.steps)
    p.use_graphs(False)
    p.select_plan(inst.n, rv, cv)
    p.select_adjoint_plan(inst.n, arv, acv)
    p.gen_screens()
    p.set_theta(0, inst.theta)
    u0 = torch.from_numpy(W.initial_field(inst)).cuda()
    tgt = torch.from_numpy(W.synthetic_target(inst, 5)).cuda()
    p.set_field(0, u0)
    p.forward_record(args.steps)
    p.fluence_loss(0, tgt)
    p.backward()
    p.synchronize()
    p.close()
    print(f"march: 4096^2, {args.steps} steps forward + adjoint, variants row {rv} col {cv} "
          f"adjoint row {arv} col {acv}; copy bytes {8 * inst.n * inst.n}", flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--out", default=None)
    ap.add_argument("--large", action="store_true",
                    help="the 4096^2 large-aperture beam (Kerr, MPA, plasma; no screens) "
                         "instead of the 1024^2 one, without the finite-difference march")
    ap.add_argument("--march", default=None, metavar="ROW,COL,ROWADJ,COLADJ",
                    help="instead: the 4096^2 forward + adjoint with these tile variants")
    ap.add_argument("--summarise", nargs=2, metavar=("FETCH", "WRITE"), default=None,
                    help="instead: summarise two rocprofv3 counter CSVs (FETCH_SIZE, "
                         "WRITE_SIZE) of a --march run into the JSON at --out")
    ap.add_argument("--copy-bytes", type=float, default=8.0 * 4096 * 4096)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    if args.summarise:
        info = summarise(args.summarise[0], args.summarise[1], args.copy_bytes,
                         args.out or "traffic.json")
        print(json.dumps(info, indent=1))
        return 0
    if args.march:
        return run_march(args)
    import dataclasses

    import workloads as W
    from .march import Propagator, desc_of, plan_variants

    if args.large:
        base = W.config5()[0]
        inst = dataclasses.replace(base, medium=dataclasses.replace(base.medium, terms=W.KPM),
                                   n_screens=0)
    else:
        inst = W.config2()[0]
    n = inst.n
    p = Propagator([desc_of(inst)], precision=args.precision, max_steps=args.steps,
                   ckpt_every=args.steps)
    p.use_graphs(False)
    u0 = W.initial_field(inst)
    n_row, n_col = plan_variants(n, args.precision)
    order = []
    for kind, count in (("row", n_row), ("col", n_col)):
        for v in range(count):
            p.select_plan(n, v if kind == "row" else 0, v if kind == "col" else 0)
            p.set_field(0, u0)
            p.forward_record(args.steps)
            p.synchronize()
            order.append([kind, v])
            print(f"{kind} variant {v}: {args.steps} steps", flush=True)
    if not args.large:
        # the finite-difference scheme's passes (variant 0 plans): one starting
        # row pass, then per step FD_ITERS column passes and as many row passes
        p.select_plan(n, 0, 0)
        p.set_finite_difference(FD_ITERS)
        p.set_field(0, u0)
        p.propagate(args.steps)
        p.synchronize()
        order.append(["fd", 0])
        print(f"finite differences: {args.steps} steps, {FD_ITERS} iterations", flush=True)
    p.close()
    info = {"grid": n, "precision": args.precision, "steps": args.steps,
            "n_row": n_row, "n_col": n_col, "order": order, "fd_iters": FD_ITERS,
            "copy_bytes": n * n * (8 if args.precision == 32 else 16),
            "source_hash": kernel_source_hash()}
    if args.out:
        with open(args.out, "w") as f:
            json.dump(info, f, indent=1)
    print("done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
