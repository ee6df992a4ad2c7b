"""Short eager marches of every compiled tile variant, for hardware counters.

    python -m paper_2306_15678_amd.passprof [--precision 32] [--steps 4] [--large]

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
                "pass_col_f32.hip", "pass_col_f64.hip")


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


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--out", default=None)
    ap.add_argument("--large", action="store_true",
                    help="the 4096^2 large-aperture beam (Kerr, MPA, plasma; no screens) "
                         "instead of the 1024^2 one, without the finite-difference march")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
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
