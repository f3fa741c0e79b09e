"""Marching Tetrahedra on the GPU: the triangle mesh of the SDF's zero level
set on the tet grid (the mesh extraction of Sec. 4.1)."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import check
from .regularizers import MeshEdges


def marching_tets(verts: torch.Tensor, sdf: torch.Tensor, tets: torch.Tensor, edges: MeshEdges | None = None,
                  vert_capacity: int | None = None, tri_capacity: int | None = None):
    """(vertices [Nv,3] float32, triangles [Nt,3] int32) on the device.
    Reads the two counts back (one synchronisation)."""
    verts, sdf, tets = verts.contiguous(), sdf.contiguous(), tets.contiguous()
    V, K = int(verts.shape[0]), int(tets.shape[0])
    if edges is None:
        edges = MeshEdges(tets, V)
    dev = verts.device
    vcap = edges.capacity if vert_capacity is None else int(vert_capacity)
    tcap = 2 * K if tri_capacity is None else int(tri_capacity)
    out_v = torch.empty((max(1, vcap), 3), dtype=torch.float32, device=dev)
    out_t = torch.empty((max(1, tcap), 3), dtype=torch.int32, device=dev)
    counts = torch.zeros(2, dtype=torch.int32, device=dev)
    n = C.c_size_t(0)
    check(_lib.lib().render_marching_tets_workspace_size(K, edges.capacity, C.byref(n)))
    ws = torch.empty(max(1, int(n.value)), dtype=torch.uint8, device=dev)
    check(_lib.lib().render_marching_tets(verts.data_ptr(), tets.data_ptr(), sdf.data_ptr(), V, K,
                                          edges.buffer.data_ptr(), edges.count.data_ptr(), edges.capacity,
                                          out_v.data_ptr(), vcap, out_t.data_ptr(), tcap, counts.data_ptr(),
                                          ws.data_ptr(), int(n.value), torch.cuda.current_stream(dev).cuda_stream))
    nv, nt = (int(x) for x in counts.cpu())
    if nv > vcap or nt > tcap:
        raise RuntimeError(f"marching tets needs {nv} vertices / {nt} triangles, capacities {vcap} / {tcap}")
    return out_v[:nv], out_t[:nt]
