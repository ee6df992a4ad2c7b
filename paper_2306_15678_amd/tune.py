"""Autotuner of the FFT tile variants (points per thread, lines per
workgroup) of the row and column passes.

For every grid size present in a ``Propagator`` it times each compiled
variant of the forward row pass and of the forward column pass with the
library's HIP-event timing hook (``ssfm_time_passes``: launches on the
context's stream), keeps the fastest of each and selects them.  Results are
cached in a JSON file keyed by device name, grid size and precision
(``SSFM_TUNE_CACHE``, default ``~/.cache/ssfm_tune.json``).
"""
from __future__ import annotations

import json
import os
from typing import Dict

import torch

from . import _lib as L
from .march import Propagator, plan_variants


def _cache_path() -> str:
    return os.environ.get("SSFM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ssfm_tune.json"))


def _key(n: int, precision: int) -> str:
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return f"{name}|n={n}|fp{precision}"


def load_cache() -> Dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(d: Dict) -> None:
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def _select(prop: Propagator, n: int, row: int, col: int) -> bool:
    """Select a variant pair; False if this precision does not build it."""
    try:
        prop.select_plan(n, row, col)
    except L.SsfmError as e:
        if e.status != L.EUNSUPPORTED:
            raise
        return False
    return True


def _tune_adjoint(prop: Propagator, n: int, n_row: int, n_col: int, reps: int) -> Dict:
    """Adjoint-pass variants for size n among those with the forward
    variants' tiling (the library refuses the others)."""
    rows, cols = [], []
    for v in range(n_row):
        try:
            prop.select_adjoint_plan(n, v, -1)
        except L.SsfmError as e:
            if e.status not in (L.EINVAL, L.EUNSUPPORTED):
                raise
            continue
        rows.append((prop.time_adjoint_passes(reps)[1], v))
    for v in range(n_col):
        try:
            prop.select_adjoint_plan(n, -1, v)
        except L.SsfmError as e:
            if e.status not in (L.EINVAL, L.EUNSUPPORTED):
                raise
            continue
        cols.append((prop.time_adjoint_passes(reps)[0], v))
    br, bc = min(rows)[1], min(cols)[1]
    prop.select_adjoint_plan(n, br, bc)
    return {"row_adj": br, "col_adj": bc, "ms_row_adj": min(rows)[0], "ms_col_adj": min(cols)[0],
            "rows_adj_ms": {v: t for t, v in rows}, "cols_adj_ms": {v: t for t, v in cols}}


def tune(prop: Propagator, reps: int = 50, use_cache: bool = True,
         verbose: bool = False) -> Dict[int, Dict]:
    """Select the fastest row and column variants for each grid size of
    ``prop`` (and, for a context that can record, the fastest adjoint-pass
    variants with the same tiling) and return the timings.  The timing
    launches write the work buffer only; the fields are unchanged."""
    cache = load_cache() if use_cache else {}
    out = {}
    for n in sorted({d.n for d in prop.descs}):
        key = _key(n, prop.precision)
        if use_cache and key in cache:
            best = cache[key]
            prop.select_plan(n, best["row"], best["col"])
            if prop.max_steps > 0 and "row_adj" in best:
                prop.select_adjoint_plan(n, best["row_adj"], best["col_adj"])
            out[n] = best
            continue
        n_row, n_col = plan_variants(n, prop.precision)
        rows, cols = [], []
        # rows vary with the column variant fixed, then the other way round;
        # a variant whose tile does not fit a workgroup at this precision is
        # not built for it (EUNSUPPORTED) and is skipped
        for v in range(n_row):
            if not _select(prop, n, v, 0):
                continue
            ms_row, _, _, _ = prop.time_passes(reps)
            rows.append((ms_row, v))
        for v in range(n_col):
            if not _select(prop, n, 0, v):
                continue
            _, ms_col, _, _ = prop.time_passes(reps)
            cols.append((ms_col, v))
        br, bc = min(rows)[1], min(cols)[1]
        prop.select_plan(n, br, bc)
        best = {"row": br, "col": bc, "ms_row": min(rows)[0], "ms_col": min(cols)[0],
                "rows_ms": [r[0] for r in rows], "cols_ms": [c[0] for c in cols]}
        if prop.max_steps > 0:
            best.update(_tune_adjoint(prop, n, n_row, n_col, reps))
        if verbose:
            print(f"tune n={n} fp{prop.precision}: rows(us)="
                  f"{[round(r[0] * 1e3, 2) for r in rows]} cols(us)="
                  f"{[round(c[0] * 1e3, 2) for c in cols]} -> row {br}, col {bc}", flush=True)
        cache[key] = best
        out[n] = best
    if use_cache:
        save_cache(cache)
    return out
