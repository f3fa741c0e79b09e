"""Coarse-to-fine pre-filtering (App. B, geometry stage).

The first pass pre-filters a cube grid over the initial domain; the box of
the kept tets' vertices (`render_prefilter_bounds`), the refitted cube around
it (`render_refit_cube`) and the rebuilt grid (`render_cube_grid`) are all
computed on the device, so the two passes need no host synchronisation.  The
SDF is the caller's: a function from vertex positions [V,3] to values [V] on
the device (in the paper, the hash-grid network), evaluated on each pass's
vertices.  This module only marshals arguments."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check
from .frontend import Params, SceneT


def _stream(dev):
    return torch.cuda.current_stream(dev).cuda_stream


def cube_grid(R: int, cube: torch.Tensor, with_tets: bool = True):
    """Kuhn grid over the device cube (lx, ly, lz, h): (verts [(R+1)^3, 3]
    float32, tets [6 R^3, 4] int32 or None)."""
    dev = cube.device
    cube = cube.float().contiguous()
    verts = torch.empty(((R + 1) ** 3, 3), dtype=torch.float32, device=dev)
    tets = torch.empty((6 * R ** 3, 4), dtype=torch.int32, device=dev) if with_tets else None
    check(_lib.lib().render_cube_grid(int(R), cube.data_ptr(), verts.data_ptr(),
                                      tets.data_ptr() if tets is not None else None, _stream(dev)))
    return verts, tets


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
                                             _stream(dev)))
    return bounds, kept


def refit_cube(bounds: torch.Tensor, cube: torch.Tensor, R: int) -> torch.Tensor:
    """The second-pass cube (device float32 [4]) around the first pass's box."""
    out = torch.empty(4, dtype=torch.float32, device=cube.device)
    check(_lib.lib().render_refit_cube(bounds.data_ptr(), cube.contiguous().data_ptr(), int(R), out.data_ptr(),
                                       _stream(cube.device)))
    return out


def coarse_to_fine(sdf_fn, R: int, s: float, params: Params | None = None, lo: float = -1.0, hi: float = 1.0,
                   device="cuda"):
    """Two-pass pre-filter over the cube [lo, hi]^3 at resolution R.  Returns
    (verts, tets, sdf, info) of the second-pass grid; info holds device
    tensors: both passes' cubes, the first pass's box and kept count."""
    params = params or Params()
    dev = torch.device(device)
    # the initial domain as the caller states it: low corner and cell size
    cube1 = torch.tensor([lo, lo, lo, float(np.float32((hi - lo) / R))], dtype=torch.float32, device=dev)
    v1, tets = cube_grid(R, cube1)
    f1 = sdf_fn(v1).float().contiguous()
    box, kept1 = prefilter_bounds(SceneT(v1, tets, f1, v1, s), params)
    cube2 = refit_cube(box, cube1, R)
    v2, _ = cube_grid(R, cube2, with_tets=False)
    f2 = sdf_fn(v2).float().contiguous()
    info = {"cube1": cube1, "pass1_box": box, "pass1_kept": kept1, "cube": cube2}
    return v2, tets, f2, info
