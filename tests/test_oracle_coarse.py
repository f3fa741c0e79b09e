"""Pins of the coarse-to-fine oracle (App. B): the kept box of a sphere
brackets the sphere to within two cells, an off-centre sphere's box is
centred on it, a scene with nothing kept has no box, and the rebuilt cube
grid covers the box with one coarse cell of margin and uniform spacing."""
import numpy as np
import pytest

import synth
from oracle import coarse


def _sphere(R, c, r):
    verts, tets = synth.kuhn_grid(R)
    sdf = np.linalg.norm(verts - np.asarray(c), axis=1) - r
    return verts.astype(np.float32), tets, sdf.astype(np.float32)


@pytest.mark.parametrize("c,r", [((0, 0, 0), 0.5), ((0.2, -0.1, 0.15), 0.3)])
def test_kept_box_brackets_the_sphere(c, r):
    R, s = 16, 2000.0
    h = 2.0 / R
    v, t, f = _sphere(R, c, r)
    lo, hi, n = coarse.kept_bounds(v, t, f, s)
    c = np.asarray(c)
    assert n > 0
    assert np.all(lo <= c - r) and np.all(hi >= c + r)
    assert np.all(lo >= c - r - 2 * h) and np.all(hi <= c + r + 2 * h)
    assert np.all(np.abs((lo + hi) / 2 - c) <= h)


def test_nothing_kept_has_no_box():
    v, t, f = _sphere(8, (0, 0, 0), 0.5)
    lo, hi, n = coarse.kept_bounds(v, t, np.full_like(f, 3.0), 320.0)
    assert lo is None and hi is None and n == 0


def test_rebuilt_grid_covers_the_box():
    R = 16
    lo, hi = np.array([-0.3, -0.2, 0.1], np.float32), np.array([0.4, 0.25, 0.3], np.float32)
    low, h = coarse.resized_cube(lo, hi, R, 2.0 / 16)
    side = float(h) * R
    assert side == pytest.approx(0.7 + 2 * 0.125, rel=1e-6)
    assert np.all(low <= lo) and np.all(low + side >= hi)
    np.testing.assert_allclose((low + side / 2), (lo + hi) / 2, atol=1e-6)
    g = coarse.grid_vertices(low, h, R)
    assert g.shape == ((R + 1) ** 3, 3) and g.dtype == np.float32
    # vertex (x, y, z) = x + (R+1)(y + (R+1) z) sits at low + (x, y, z) h
    for x, y, z in [(0, 0, 0), (R, 0, 0), (3, 5, 7), (R, R, R)]:
        np.testing.assert_allclose(g[x + (R + 1) * (y + (R + 1) * z)], low + np.array([x, y, z]) * float(h),
                                   atol=1e-6)
    d = np.diff(g[: R + 1, 0].astype(np.float64))
    assert np.allclose(d, float(h), atol=1e-6)
