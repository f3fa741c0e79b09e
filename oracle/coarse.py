"""Oracle of the coarse-to-fine pre-filter (App. B, geometry stage).  Test
infrastructure only.

The first pass pre-filters the tets of a cube grid (the oracle's own
pre-filter, Sec. 3.2); the bounding box of the kept tets' vertices is taken;
the grid is rebuilt over that box and the SDF sampled at the new vertices for
the second pass.

Readings (listed with the rest of the paper's readings): the rebuilt grid
keeps the resolution R and cubic cells: a cube centred on the box with side
= the box's largest extent plus one coarse cell on each side; vertex
coordinates are lo + i * h in float32 with h = side / R (float32), lo the
cube's low corner, for i = 0..R along each axis.  An empty kept set leaves
the grid unchanged.
"""
from __future__ import annotations

import numpy as np

from . import Geometry, params_array, prefilter


def kept_bounds(verts, tets, sdf, s: float, params=None):
    """(lo [3], hi [3], kept count) of the vertices of the kept tets, float32."""
    verts = np.asarray(verts, np.float32)
    tets = np.asarray(tets, np.int32)
    sdf = np.asarray(sdf, np.float32)
    colors = np.zeros_like(verts)
    g = Geometry(verts, tets, sdf, colors)
    P = params_array(s) if params is None else params
    keep, *_ = prefilter(g, P, prec=32)
    if not keep.any():
        return None, None, 0
    vid = np.unique(tets[keep].ravel())
    v = verts[vid]
    return v.min(0), v.max(0), int(keep.sum())


def resized_cube(lo, hi, R: int, old_h: float):
    """(cube low corner [3] float32, cell size float32) of the second-pass grid."""
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    ext = float(np.max(hi - lo))
    side = np.float32(ext + 2.0 * old_h)
    centre = (lo.astype(np.float64) + hi.astype(np.float64)) / 2.0
    low = (centre - float(side) / 2.0).astype(np.float32)
    h = np.float32(side / np.float32(R))
    return low, h


def grid_vertices(low, h, R: int):
    """[(R+1)^3, 3] float32, vertex x + (R+1)(y + (R+1) z) at low + (x, y, z) * h."""
    i = np.arange(R + 1, dtype=np.float32)
    ax = [np.float32(low[a]) + i * np.float32(h) for a in range(3)]
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float32)
