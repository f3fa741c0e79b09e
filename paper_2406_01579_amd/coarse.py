"""Coarse-to-fine pre-filtering (App. B, geometry stage).

The first pass pre-filters a cube grid over the initial domain; the box of the kept
tets' vertices comes from the GPU (`render_prefilter_bounds`); the grid is
rebuilt at the same resolution over a cube around that box (side = the box's
largest extent plus one coarse cell on each side) and the SDF is sampled at
the new vertices for the second pass, which is the ordinary forward's pre-filter.
The SDF is the caller's: a function from vertex positions [V,3] to values [V]
on the device (in the paper, the hash-grid network)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check
from .frontend import Params, SceneT

# the six axis orders of a cube's Kuhn split, in lexicographic order
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_grid(R: int, low, h, device="cuda"):
    """Cube grid of R^3 cells with low corner `low` and cell size h (float32):
    vertex (x, y, z) has index x + (R+1)(y + (R+1) z) and sits at low + (x, y, z) h;
    cell q = x + R(y + R z) is split into tets 6q + p, p over the axis orders,
    with vertices (v0, v0 + e_a, v0 + e_a + e_b, v0 + (1, 1, 1))."""
    dev = torch.device(device)
    n = R + 1
    i = torch.arange(n, device=dev, dtype=torch.float32)
    ax = [torch.tensor(float(np.float32(low[a])), device=dev) + i * torch.tensor(float(np.float32(h)), device=dev)
          for a in range(3)]
    zz, yy, xx = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    verts = torch.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], 1).contiguous()
    c = torch.arange(R, device=dev, dtype=torch.int64)
    cz, cy, cx = torch.meshgrid(c, c, c, indexing="ij")
    stride = (1, n, n * n)
    v0 = (cx + n * (cy + n * cz)).reshape(-1)
    tets = torch.empty((R ** 3, 6, 4), dtype=torch.int64, device=dev)
    for p, (a, b, _) in enumerate(_PERMS):
        s1 = stride[a]
        s2 = s1 + stride[b]
        tets[:, p, 0] = v0
        tets[:, p, 1] = v0 + s1
        tets[:, p, 2] = v0 + s2
        tets[:, p, 3] = v0 + 1 + n + n * n
    return verts, tets.reshape(-1, 4).to(torch.int32).contiguous()


def prefilter_bounds(scene: SceneT, params: Params | None = None):
    """(bounds [6] float32 device tensor: min xyz, max xyz -- NaN if nothing
    is kept; kept count [1] int64 device tensor)."""
    params = params or Params()
    dev = scene.verts.device
    bounds = torch.empty(6, dtype=torch.float32, device=dev)
    kept = torch.empty(1, dtype=torch.int64, device=dev)
    sc = _lib.render_scene(scene.verts.data_ptr(), scene.tets.data_ptr(), scene.sdf.data_ptr(), None,
                           int(scene.verts.shape[0]), int(scene.tets.shape[0]), float(scene.s))
    pc = params.c()
    check(_lib.lib().render_prefilter_bounds(C.byref(sc), C.byref(pc), bounds.data_ptr(), kept.data_ptr(),
                                             torch.cuda.current_stream(dev).cuda_stream))
    return bounds, kept


def resized_cube(lo, hi, R: int, old_h: float):
    """(low corner [3] float32, cell size float32) of the second-pass cube grid."""
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    side = np.float32(float(np.max(hi - lo)) + 2.0 * old_h)
    centre = (lo.astype(np.float64) + hi.astype(np.float64)) / 2.0
    low = (centre - float(side) / 2.0).astype(np.float32)
    return low, np.float32(side / np.float32(R))


def coarse_to_fine(sdf_fn, R: int, s: float, params: Params | None = None, lo: float = -1.0, hi: float = 1.0,
                   device="cuda"):
    """Two-pass pre-filter.  Returns (verts, tets, sdf, info) of the second-pass
    grid; info holds both passes' boxes and kept counts.  One host read of the
    first-pass box."""
    params = params or Params()
    low1 = np.full(3, lo, np.float32)
    h1 = np.float32((hi - lo) / R)
    v1, t1 = kuhn_grid(R, low1, h1, device)
    f1 = sdf_fn(v1).float().contiguous()
    b, k = prefilter_bounds(SceneT(v1, t1, f1, v1, s), params)
    box = b.cpu().numpy()
    kept1 = int(k.item())
    info = {"pass1_box": box, "pass1_kept": kept1}
    if kept1 == 0 or not np.all(np.isfinite(box)):
        return v1, t1, f1, info
    low2, h2 = resized_cube(box[:3], box[3:], R, float(h1))
    v2, t2 = kuhn_grid(R, low2, h2, device)
    f2 = sdf_fn(v2).float().contiguous()
    info.update(low=low2, h=float(h2))
    return v2, t2, f2, info
