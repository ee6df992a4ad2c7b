"""Beam diagnostics of the paper's evaluation: hot-area count and moments.

Test infrastructure, like the rest of ``oracle/``: plain FP64 numpy, used
only by the tests and the bench's CPU baseline.

* Hot areas (Results, multiple filamentation and the turbulent-path
  experiment): a hot area is a closed region of the fluence where w >= w_p;
  N_ha is their number.  Regions are 4-connected (pixels sharing an edge),
  and on the periodic grid of the march a region may continue across the
  window edge (``periodic=True``).
* Spatial moments (Eq. (8), printed garbled): Q(p, m) = sum w^p
  (x^2 + y^2)^m dx^2 over the cell-centred grid, x_j = (j + 1/2 - N/2) dx;
  the printed exponents read as p = 2m, the usual energy moments are p = 1.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def hot_mask(w: np.ndarray, threshold: float) -> np.ndarray:
    """Pixels of a hot area: w >= w_p."""
    return w >= threshold


def hot_area_count(w: np.ndarray, threshold: float, periodic: bool = True) -> int:
    """Number of 4-connected regions with w >= threshold.

    scipy's labelling (a library primitive) labels the regions of the open
    window; with ``periodic`` the labels that touch across the last/first
    row and column are then merged with a small union-find over labels.
    """
    mask = hot_mask(w, threshold)
    lab, n = ndimage.label(mask, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    if n == 0 or not periodic:
        return int(n)
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    def join(a, b):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)

    for a, b in zip(lab[-1, :], lab[0, :]):      # bottom row meets top row
        if a and b:
            join(int(a), int(b))
    for a, b in zip(lab[:, -1], lab[:, 0]):      # right column meets left column
        if a and b:
            join(int(a), int(b))
    return len({find(k) for k in range(1, n + 1)})


def flood_fill_count(mask: np.ndarray, periodic: bool = True) -> int:
    """Brute-force count by breadth-first flood fill (small grids only)."""
    ny, nx = mask.shape
    seen = np.zeros_like(mask, dtype=bool)
    count = 0
    for y0 in range(ny):
        for x0 in range(nx):
            if not mask[y0, x0] or seen[y0, x0]:
                continue
            count += 1
            stack = [(y0, x0)]
            seen[y0, x0] = True
            while stack:
                y, x = stack.pop()
                for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    yy, xx = y + dy, x + dx
                    if periodic:
                        yy %= ny
                        xx %= nx
                    elif not (0 <= yy < ny and 0 <= xx < nx):
                        continue
                    if mask[yy, xx] and not seen[yy, xx]:
                        seen[yy, xx] = True
                        stack.append((yy, xx))
    return count


def grid_r2(n: int, length: float) -> np.ndarray:
    """x^2 + y^2 on the cell-centred grid [y, x]."""
    dx = length / n
    x = (np.arange(n) + 0.5 - n / 2) * dx
    return x[None, :] ** 2 + x[:, None] ** 2


def moment(w: np.ndarray, length: float, p: float, m: int) -> float:
    """Q(p, m) = sum w^p (x^2 + y^2)^m dx^2 (FP64)."""
    n = w.shape[0]
    dx = length / n
    return float(np.sum(w.astype(np.float64) ** p * grid_r2(n, length) ** m) * dx * dx)


# ------------------------------------------------------- measure vector
# The GA's fitness (Math and Equations, GA paragraph): a vector P that
# characterises a solution, compared with the dense-grid solution's P0 by
# the Euclidean metric.  P is read here as the fluence's integral
# quantities that the text names: its energy and the Eq. (8) spatial
# moments (the printed m = 1 moment, w^2 r^2, and the usual energy moments),
# its peak (the on-axis intensity the text monitors) and the hot-area count.
MEASURE_NAMES = ("energy Q(1,0)", "Q(1,1)", "Q(2,0)", "Q(2,1)", "peak", "hot areas")


def measure_vector(w: np.ndarray, length: float, w_p: float, periodic: bool = True) -> np.ndarray:
    """P = (Q(1,0), Q(1,1), Q(2,0), Q(2,1), max w, N_ha(w >= w_p))."""
    return np.array([moment(w, length, 1.0, 0), moment(w, length, 1.0, 1),
                     moment(w, length, 2.0, 0), moment(w, length, 2.0, 1),
                     float(np.max(w)), float(hot_area_count(w, w_p, periodic))])


def measure_distance(p: np.ndarray, p0: np.ndarray) -> float:
    """Euclidean distance of P from P0 in component-wise relative units:
    sqrt(sum_k ((P_k - P0_k) / s_k)^2), s_k = |P0_k| (1 where P0_k = 0), so
    that quantities of different units and sizes weigh alike."""
    p = np.asarray(p, dtype=np.float64)
    p0 = np.asarray(p0, dtype=np.float64)
    s = np.where(p0 != 0.0, np.abs(p0), 1.0)
    return float(np.sqrt(np.sum(((p - p0) / s) ** 2)))
