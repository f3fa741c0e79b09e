"""Graph-captured rendering steps.

The forward and backward launch sequences are pure kernel launches on one
stream: descriptors travel as kernel arguments, every data-dependent size
stays on the device, and buffers are sized by capacities with a device
overflow flag.  So a whole training step -- forward through the autograd
Function and its backward -- can be captured once in a HIP graph and then
replayed with no host work per step.  Inputs are static tensors: copy new
values into ``step.verts`` / ``step.sdf`` / ``step.colors`` (and the upstream
gradient into ``step.dout``) before ``replay()``.  After a replay,
``check()`` reads the overflow flag; if the data outgrew the capacities the
step must be re-captured with larger ones (``recapture()``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .frontend import Params, Renderer, TetSplatFunction


class CapturedStep:
    """out = render(verts, sdf, colors) for fixed tets and cameras; loss
    gradient dout; gradients land in ``verts.grad``, ``sdf.grad``,
    ``colors.grad`` (tensors owned by the graph, overwritten per replay)."""

    def __init__(self, verts, sdf, colors, tets, cams, s, params: Params | None = None, dout=None,
                 margin: float = 1.5, warmup: int = 2, device="cuda"):
        self.device = torch.device(device)
        self.params = params or Params()
        self.cams = np.asarray(cams, np.float32)
        self.s = float(s)
        self.margin = margin
        self.tets = tets.to(self.device).int().contiguous()
        self.verts = verts.detach().to(self.device).float().clone().requires_grad_(True)
        self.sdf = sdf.detach().to(self.device).float().clone().requires_grad_(True)
        self.colors = colors.detach().to(self.device).float().clone().requires_grad_(True)
        nv = self.cams.shape[0]
        W, H = int(self.cams[0, 0]), int(self.cams[0, 1])
        self.dout = torch.zeros((nv, 8, H, W), device=self.device) if dout is None else dout.detach().clone()
        self._capture(warmup, margin)

    # ------------------------------------------------------------------
    def _size(self, margin):
        """Exact capacities from an eager forward, with headroom."""
        probe = Renderer(self.params, device=self.device, check="sync")
        from .frontend import SceneT
        sc = SceneT(self.verts.detach(), self.tets, self.sdf.detach(), self.colors.detach(), self.s)
        plan = probe.forward([sc], self.cams)
        st = plan.status
        kept = int(int(st.kept) * margin) + 1024
        ent = int(int(st.entries_needed) * margin) + 4096
        del plan
        return kept, ent

    def _body(self):
        for t in (self.verts, self.sdf, self.colors):
            t.grad = None
        out = TetSplatFunction.apply(self.verts, self.sdf, self.colors, self.tets, self.cams, self.s, self.renderer)
        torch.autograd.backward(out, self.dout)
        return out

    def _fresh_leaves(self):
        # new leaf tensors, so their gradient accumulators are created on the
        # stream that runs the next backward
        self.verts = self.verts.detach().clone().requires_grad_(True)
        self.sdf = self.sdf.detach().clone().requires_grad_(True)
        self.colors = self.colors.detach().clone().requires_grad_(True)

    def _capture(self, warmup, margin):
        kept, ent = self._size(margin)
        self.kept_cap, self.entry_cap = kept, ent
        self.renderer = Renderer(self.params, device=self.device, check="none")
        from .frontend import SceneT
        sc = SceneT(self.verts.detach(), self.tets, self.sdf.detach(), self.colors.detach(), self.s)
        self.renderer.set_capacity([sc], self.cams, None, kept, ent)
        self._fresh_leaves()
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            for _ in range(max(1, warmup)):
                self._body()
        torch.cuda.current_stream(self.device).wait_stream(side)
        torch.cuda.synchronize(self.device)
        self._fresh_leaves()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.out = self._body()
        self.plan = self.renderer.last_plan
        torch.cuda.synchronize(self.device)

    # ------------------------------------------------------------------
    def replay(self):
        self.graph.replay()
        return self.out.detach()

    @property
    def grads(self):
        return self.verts.grad, self.sdf.grad, self.colors.grad

    def check(self) -> _lib.render_status:
        """Synchronise and read the captured forward's counters; raises if a
        capacity was exceeded (outputs of that replay are invalid)."""
        st = self.renderer.read_status(self.plan)
        if st.overflow:
            from .frontend import CapacityError
            raise CapacityError("captured step exceeded its capacities; call recapture()")
        return st

    def recapture(self, margin: float | None = None):
        self.graph = None
        self._capture(2, margin or 2.0 * self.margin)
