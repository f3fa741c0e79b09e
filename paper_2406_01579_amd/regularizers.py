"""Eikonal and normal-consistency regularisers (Sec. 4.2) on the GPU.

``MeshEdges(tets, V)`` builds the unique-edge list of the tet mesh once per
topology; ``regularizers(verts, sdf, tets, edges)`` returns (L_eik, L_nc) as
float64 device scalars and is differentiable with respect to ``verts`` and
``sdf`` (its backward runs the kernels again with the upstream gradients as
the two weights, read on the device: no host synchronisation)."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import check


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class MeshEdges:
    """Unique (a < b) edges of a tet mesh in ascending order, on the device."""

    def __init__(self, tets: torch.Tensor, V: int):
        tets = tets.contiguous()
        assert tets.dtype == torch.int32 and tets.is_cuda and tets.dim() == 2 and tets.shape[1] == 4
        K = int(tets.shape[0])
        dev = tets.device
        n = C.c_size_t(0)
        check(_lib.lib().render_mesh_edges_workspace_size(K, C.byref(n)))
        ws = torch.empty(max(1, int(n.value)), dtype=torch.uint8, device=dev)
        self.buffer = torch.empty((max(1, 6 * K), 2), dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        check(_lib.lib().render_mesh_edges(tets.data_ptr(), K, int(V), self.buffer.data_ptr(), self.count.data_ptr(),
                                           ws.data_ptr(), int(n.value), _stream(dev)))
        self.V = int(V)
        self._ws = ws

    @property
    def edges(self) -> torch.Tensor:
        """[E, 2] view (reads the count: synchronises)."""
        return self.buffer[: int(self.count.item())]

    @property
    def capacity(self) -> int:
        return int(self.buffer.shape[0])


def _run(verts, sdf, tets, edges: MeshEdges, weights=None, dverts=None, dsdf=None):
    V, K = int(verts.shape[0]), int(tets.shape[0])
    n = C.c_size_t(0)
    check(_lib.lib().render_regularizers_workspace_size(V, K, C.byref(n)))
    ws = torch.empty(max(1, int(n.value)), dtype=torch.uint8, device=verts.device)
    losses = torch.empty(2, dtype=torch.float64, device=verts.device)
    ptr = (lambda t: None if t is None else t.data_ptr())
    check(_lib.lib().render_regularizers(verts.data_ptr(), tets.data_ptr(), sdf.data_ptr(), V, K,
                                         edges.buffer.data_ptr(), edges.count.data_ptr(), edges.capacity,
                                         ptr(weights), losses.data_ptr(), ptr(dverts), ptr(dsdf), ws.data_ptr(),
                                         int(n.value), _stream(verts.device)))
    return losses


class RegularizerFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, verts, sdf, tets, edges):
        v, f = verts.detach().contiguous(), sdf.detach().contiguous()
        t = tets.contiguous()
        ctx.save_for_backward(v, f, t)
        ctx.edges = edges
        return _run(v, f, t, edges)

    @staticmethod
    def backward(ctx, g):
        v, f, t = ctx.saved_tensors
        w = g.detach().float().contiguous()
        dv = torch.zeros_like(v)
        df = torch.zeros_like(f)
        _run(v, f, t, ctx.edges, w, dv, df)
        return dv, df, None, None


def regularizers(verts, sdf, tets, edges: MeshEdges) -> torch.Tensor:
    """(L_eik, L_nc) as a float64 [2] device tensor."""
    return RegularizerFunction.apply(verts, sdf, tets, edges)
