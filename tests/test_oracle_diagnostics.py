"""Pins of the oracle's hot-area count and spatial moments."""
import math

import numpy as np
import pytest

from oracle import diagnostics as D


def _count(mask, periodic=True):
    return D.hot_area_count(mask.astype(np.float64), 0.5, periodic)


def test_simple_shapes():
    z = np.zeros((16, 16))
    assert _count(z) == 0
    assert _count(np.ones((16, 16))) == 1
    a = z.copy()
    a[2:5, 2:5] = 1
    a[8:12, 9:13] = 1
    assert _count(a) == 2
    # squares touching only at a corner are separate under 4-connectivity
    b = z.copy()
    b[2:5, 2:5] = 1
    b[5:8, 5:8] = 1
    assert _count(b) == 2
    # a ring is one region; its hole is not a region
    yy, xx = np.mgrid[0:16, 0:16]
    r = np.hypot(yy - 7.5, xx - 7.5)
    assert _count((r > 3) & (r < 6)) == 1
    # a U shape is one region
    u = z.copy()
    u[3:12, 3] = 1
    u[3:12, 10] = 1
    u[11, 3:11] = 1
    assert _count(u) == 1


def test_checkerboard_cells_are_isolated():
    yy, xx = np.mgrid[0:8, 0:8]
    board = (yy + xx) % 2 == 0
    assert _count(board, periodic=False) == 32
    assert _count(board, periodic=True) == 32


def test_periodic_wrap():
    z = np.zeros((12, 12))
    edge = z.copy()
    edge[4:7, 0:2] = 1
    edge[4:7, 10:12] = 1
    assert _count(edge, periodic=True) == 1
    assert _count(edge, periodic=False) == 2
    corner = z.copy()
    corner[0:2, 0:2] = corner[0:2, 10:12] = corner[10:12, 0:2] = corner[10:12, 10:12] = 1
    assert _count(corner, periodic=True) == 1
    assert _count(corner, periodic=False) == 4
    stripes = z.copy()
    stripes[2, :] = 1
    stripes[6, :] = 1
    assert _count(stripes, periodic=True) == 2


def test_threshold_is_inclusive():
    w = np.zeros((8, 8))
    w[2, 2] = 0.5
    w[5, 5] = 0.4999999999999999
    assert D.hot_area_count(w, 0.5) == 1


@pytest.mark.parametrize("shape,density,periodic", [
    ((7, 9), 0.45, False), ((7, 9), 0.45, True), ((16, 16), 0.5, True),
    ((24, 24), 0.55, True), ((24, 24), 0.3, False), ((13, 20), 0.6, True)])
def test_against_brute_force_flood_fill(shape, density, periodic):
    rng = np.random.default_rng(hash((shape, density, periodic)) % 2**32)
    for _ in range(20):
        mask = rng.random(shape) < density
        assert _count(mask, periodic) == D.flood_fill_count(mask, periodic)


def test_moments_of_a_gaussian():
    """w = I0 exp(-2 r^2/w0^2): Q(1,0) = P = pi I0 w0^2/2, Q(1,1) = P w0^2/2,
    Q(2,1) = pi I0^2 w0^4/16 (grid sum of a well-resolved Gaussian)."""
    n, length, w0, i0 = 256, 8e-3, 0.6e-3, 3e15
    w = i0 * np.exp(-2 * D.grid_r2(n, length) / w0 ** 2)
    p = math.pi * i0 * w0 ** 2 / 2
    assert D.moment(w, length, 1, 0) == pytest.approx(p, rel=1e-12)
    assert D.moment(w, length, 1, 1) == pytest.approx(p * w0 ** 2 / 2, rel=1e-12)
    assert D.moment(w, length, 2, 1) == pytest.approx(math.pi * i0 ** 2 * w0 ** 4 / 16, rel=1e-12)
    assert D.moment(w, length, 0, 0) == pytest.approx(length ** 2, rel=1e-14)


def test_measure_vector_of_a_gaussian():
    """Closed forms of the fluence w = I0 exp(-2 r^2 / w0^2) on a window
    wide enough to hold it (int_0^inf r^3 exp(-a r^2) dr = 1 / (2 a^2)):
    energy pi w0^2 I0 / 2, Q(1,1) = pi w0^4 I0 / 4, Q(2,0) = pi w0^2 I0^2 / 4,
    Q(2,1) = pi w0^4 I0^2 / 16, peak I0 (the grid
    is cell-centred, so the peak sample sits half a cell off axis: I0
    exp(-dx^2 / w0^2)), one hot area above half the peak."""
    n, length, w0, i0 = 256, 8e-3, 1e-3, 3e16
    r2 = D.grid_r2(n, length)
    w = i0 * np.exp(-2 * r2 / w0 ** 2)
    p = D.measure_vector(w, length, 0.5 * i0)
    dx = length / n
    want = [np.pi * w0 ** 2 * i0 / 2, np.pi * w0 ** 4 * i0 / 4, np.pi * w0 ** 2 * i0 ** 2 / 4,
            np.pi * w0 ** 4 * i0 ** 2 / 16, i0 * np.exp(-dx ** 2 / w0 ** 2), 1.0]
    assert np.allclose(p, want, rtol=1e-10, atol=0)
    assert D.MEASURE_NAMES[0].startswith("energy") and len(D.MEASURE_NAMES) == len(p)


def test_measure_distance_by_hand():
    """Relative Euclidean distance: equal vectors 0; one component doubled
    1; two components each 10 % off sqrt(0.02); a zero reference component
    counts absolutely; scaling P and P0 together leaves d."""
    p0 = np.array([2.0, 4.0, 8.0, 16.0, 1.0, 3.0])
    assert D.measure_distance(p0, p0) == 0.0
    p = p0.copy()
    p[2] *= 2
    assert D.measure_distance(p, p0) == pytest.approx(1.0, rel=1e-15)
    p = p0.copy()
    p[0] *= 1.1
    p[5] *= 0.9
    assert D.measure_distance(p, p0) == pytest.approx(np.sqrt(0.02), rel=1e-14)
    z = np.array([1.0, 0.0])
    assert D.measure_distance(np.array([1.0, 0.5]), z) == pytest.approx(0.5, rel=1e-15)
    assert D.measure_distance(7 * p, 7 * p0) == pytest.approx(D.measure_distance(p, p0), rel=1e-14)
