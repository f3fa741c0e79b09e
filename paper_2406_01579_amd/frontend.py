"""PyTorch front end of the gfx950 tetrahedron rasterizer.

PyTorch supplies device memory and the stream; all rendering work happens in
the HIP kernels behind the C ABI (include/tetsplat.h).  This module only
builds the ABI's argument structs from tensors, sizes and owns workspaces,
and wraps the forward/backward pair in a torch.autograd.Function.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import check

CAM_FIELDS = 22


@dataclass
class Params:
    """Blending and tiling parameters.  The thresholds are the ones of the
    3DGS rasterizer the paper builds on (Sec. 3.3); prefilter_tf is the
    paper's T_f (Sec. 3.2)."""
    tile_w: int = 8
    tile_h: int = 8
    alpha_min: float = 1.0 / 255.0
    alpha_clamp: float = 0.99
    t_min: float = 1e-4
    prefilter_tf: float = 1.0 / 255.0
    recompute_state: bool = False   # no per-pixel state in the workspace; the backward recomputes it
    waves: int = 4   # waves sharing one 8x8 tile
    window: int = 0  # per-pixel resort window N_w (Sec. 3.3); 0: per-tile order
    deterministic: bool = False     # bitwise-reproducible gradients (fixed-order sums)
    record_grads: bool = False      # one gradient accumulator per record instead of per entry
    chunk_fwd: int = 0   # entries per LDS step of the forward's tile walk (32, 64; 0: 64), multi-wave 8x8 only
    chunk_bwd: int = 0   # the same for the backward (16, 32; 0: 32)

    def flags(self) -> int:
        return ((_lib.RENDER_RECOMPUTE_STATE if self.recompute_state else 0) |
                (_lib.RENDER_DETERMINISTIC if self.deterministic else 0) |
                (_lib.RENDER_RECORD_GRADS if self.record_grads else 0))

    def c(self) -> _lib.render_params:
        return _lib.render_params(self.tile_w, self.tile_h, self.flags(), self.waves,
                                  self.alpha_min, self.alpha_clamp, self.t_min, self.prefilter_tf, self.window,
                                  self.chunk_fwd, self.chunk_bwd)

    @classmethod
    def exact(cls, **kw):
        """Thresholds off: the rendered function is piecewise smooth."""
        d = dict(alpha_min=0.0, alpha_clamp=1.0, t_min=0.0)
        d.update(kw)
        return cls(**d)


@dataclass
class SceneT:
    """Device tensors of one scene (float32 / int32, contiguous)."""
    verts: torch.Tensor
    tets: torch.Tensor
    sdf: torch.Tensor
    colors: torch.Tensor
    s: float

    @classmethod
    def from_numpy(cls, scene, device="cuda"):
        return cls(torch.as_tensor(scene.verts, device=device).float().contiguous(),
                   torch.as_tensor(scene.tets, device=device).int().contiguous(),
                   torch.as_tensor(scene.sdf, device=device).float().contiguous(),
                   torch.as_tensor(scene.colors, device=device).float().contiguous(),
                   float(scene.s))

    def c(self) -> _lib.render_scene:
        for t in (self.verts, self.tets, self.sdf, self.colors):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("scene tensors must be contiguous device tensors")
        assert self.verts.dtype == torch.float32 and self.sdf.dtype == torch.float32
        assert self.colors.dtype == torch.float32 and self.tets.dtype == torch.int32
        return _lib.render_scene(self.verts.data_ptr(), self.tets.data_ptr(), self.sdf.data_ptr(),
                                 self.colors.data_ptr(), int(self.verts.shape[0]), int(self.tets.shape[0]),
                                 float(self.s))


def make_views(cams: np.ndarray, view_scene, outs) -> C.Array:
    cams = np.asarray(cams, np.float32)
    arr = (_lib.render_view * cams.shape[0])()
    for v in range(cams.shape[0]):
        c = cams[v]
        rv = arr[v]
        rv.scene = int(view_scene[v])
        rv.width, rv.height = int(c[0]), int(c[1])
        for k in range(9):
            rv.R[k] = float(c[2 + k])
        for k in range(3):
            rv.t[k] = float(c[11 + k])
        rv.fx, rv.fy, rv.cx, rv.cy, rv.znear = (float(x) for x in c[14:19])
        for k in range(3):
            rv.bg[k] = float(c[19 + k])
        rv.out = outs[v].data_ptr()
    return arr


class CapacityError(RuntimeError):
    pass


@dataclass
class Plan:
    """One forward's workspace and the arguments its backward must repeat."""
    scenes: list
    scene_c: C.Array
    view_c: C.Array
    params_c: _lib.render_params
    kept_cap: int
    entry_cap: int
    workspace: torch.Tensor
    outs: list
    status: _lib.render_status | None = None
    keep: list = field(default_factory=list)  # tensors the pointers refer to
    header_copy: torch.Tensor | None = None    # pinned copy of the status header (lazy check)
    header_event: object = None
    sig: tuple = ()
    stacked: torch.Tensor | None = None          # [nv, 8, H, W] when all views share a size


class Renderer:
    """Holds parameters and capacity estimates; every forward gets its own
    workspace tensor, so several forwards may await their backward.

    check="sync": every forward waits for its status (exact re-planning on a
    capacity overflow, the forward is re-run).  check="lazy": the status is
    copied to pinned memory without waiting and verified before the backward
    and at the next forward of the same shape; an overflow there raises
    CapacityError (never a silent wrong result), and the capacities are
    enlarged for later calls.  check="none": no host-side status traffic at
    all (for stream capture); the caller reads the status itself
    (read_status / CapturedStep.check)."""

    def __init__(self, params: Params | None = None, device="cuda", check: str = "sync"):
        self.params = params or Params()
        self.device = torch.device(device)
        self.check = check
        self._caps = {}
        _lib.lib()

    # -- sizing ---------------------------------------------------------------
    def _signature(self, scenes, cams, view_scene):
        return (tuple((int(s.verts.shape[0]), int(s.tets.shape[0])) for s in scenes),
                tuple((int(c[0]), int(c[1])) for c in np.asarray(cams)), tuple(int(x) for x in view_scene),
                self.params.tile_w, self.params.tile_h)

    def workspace_bytes(self, scene_c, view_c, params_c, kept_cap, entry_cap) -> int:
        n = C.c_size_t(0)
        check(_lib.lib().render_workspace_size(C.byref(scene_c), len(scene_c), C.byref(view_c), len(view_c),
                                               C.byref(params_c), kept_cap, entry_cap, C.byref(n)))
        return int(n.value)

    # -- forward ----------------------------------------------------------------
    def set_capacity(self, scenes, cams, view_scene, kept_cap: int, entry_cap: int):
        """Fix the capacities used for this shape of call (e.g. before capture)."""
        cams = np.asarray(cams, np.float32)
        if view_scene is None:
            view_scene = np.zeros(cams.shape[0], np.int32)
        self._caps[self._signature(scenes, cams, view_scene)] = (int(kept_cap), int(entry_cap))

    def capacity(self, scenes, cams, view_scene=None):
        cams = np.asarray(cams, np.float32)
        if view_scene is None:
            view_scene = np.zeros(cams.shape[0], np.int32)
        return self._caps.get(self._signature(scenes, cams, view_scene))

    def forward(self, scenes, cams, view_scene=None, stream=None, caps=None) -> Plan:
        """caps=(kept_cap, entry_cap) overrides the remembered capacities."""
        cams = np.asarray(cams, np.float32)
        nv = cams.shape[0]
        if view_scene is None:
            view_scene = np.zeros(nv, np.int32)
        sizes = {(int(c[0]), int(c[1])) for c in cams}
        if len(sizes) == 1:
            # one [nv, 8, H, W] tensor; the views are its slices
            W0, H0 = sizes.pop()
            stacked = torch.empty((nv, 8, H0, W0), device=self.device, dtype=torch.float32)
            outs = list(stacked.unbind(0))
        else:
            stacked = None
            outs = [torch.empty((8, int(c[1]), int(c[0])), device=self.device, dtype=torch.float32) for c in cams]
        scene_c = (_lib.render_scene * len(scenes))(*[s.c() for s in scenes])
        view_c = make_views(cams, view_scene, outs)
        params_c = self.params.c()
        st = torch.cuda.current_stream(self.device).cuda_stream if stream is None else stream
        sig = self._signature(scenes, cams, view_scene)
        kept_cap, entry_cap = self._caps.get(sig, (0, 0)) if caps is None else (int(caps[0]), int(caps[1]))
        if entry_cap == 0:
            # first sight of this shape: generous bound, refined after the call
            rec = sum(int(scenes[int(view_scene[v])].tets.shape[0]) for v in range(nv))
            entry_cap = max(4096, 3 * rec)
        for _attempt in range(4):
            nbytes = self.workspace_bytes(scene_c, view_c, params_c, kept_cap, entry_cap)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            check(_lib.lib().render_forward(C.byref(scene_c), len(scenes), C.byref(view_c), nv, C.byref(params_c),
                                            kept_cap, entry_cap, ws.data_ptr(), nbytes, st))
            plan = Plan(scenes, scene_c, view_c, params_c, kept_cap, entry_cap, ws, outs)
            plan.stacked = stacked
            self.last_plan = plan
            if self.check == "none":
                return plan
            if self.check != "sync" and sig in self._caps:
                self._verify_pending()
                plan.header_copy = torch.empty(_lib.STATUS_BYTES, dtype=torch.uint8, pin_memory=True)
                plan.header_copy.copy_(ws[:_lib.STATUS_BYTES], non_blocking=True)
                plan.header_event = torch.cuda.Event()
                plan.header_event.record()
                plan.sig = sig
                self._pending = plan
                return plan
            stt = self.read_status(plan, st)
            if stt.invalid_index:
                raise ValueError("a tet has a vertex index outside [0, V)")
            need_kept = int(stt.kept) + 1024
            need_ent = int(stt.entries_needed)
            if stt.overflow == 0:
                # shrink generous first guesses, keep headroom for SDF drift
                k2 = int(need_kept * 1.25)
                e2 = int(need_ent * 1.3) + 4096
                if kept_cap == 0 or entry_cap > 2 * e2:
                    self._caps[sig] = (k2, e2)
                else:
                    self._caps[sig] = (kept_cap, entry_cap)
                return plan
            kept_cap = int(need_kept * 1.25) if (stt.overflow & 1) else kept_cap
            entry_cap = int(need_ent * 1.3) + 4096 if (stt.overflow & 6) else entry_cap
            if stt.overflow & 1:
                entry_cap = max(entry_cap, 2 * entry_cap)
        raise RuntimeError("could not size the workspace")

    def _verify(self, plan: Plan):
        if plan.header_copy is None:
            return
        plan.header_event.synchronize()
        s = _lib.render_status()
        check(_lib.lib().render_decode_status(plan.header_copy.data_ptr(), C.byref(s)))
        plan.status = s
        plan.header_copy = None
        if s.overflow:
            k, e = self._caps.get(plan.sig, (0, 0))
            self._caps[plan.sig] = (int(s.kept * 1.25) + 1024 if s.overflow & 1 else k,
                                    int(s.entries_needed * 1.3) + 4096 if s.overflow & 6 else e)
            raise CapacityError("workspace capacity exceeded in a forward pass; its outputs are invalid "
                                "(capacities enlarged for the next call)")
        if s.invalid_index:
            raise ValueError("a tet has a vertex index outside [0, V)")

    def _verify_pending(self):
        p = getattr(self, "_pending", None)
        if p is not None:
            self._pending = None
            self._verify(p)

    def read_status(self, plan: Plan, stream=None) -> _lib.render_status:
        st = torch.cuda.current_stream(self.device).cuda_stream if stream is None else stream
        s = _lib.render_status()
        check(_lib.lib().render_read_status(plan.workspace.data_ptr(), C.byref(s), st))
        plan.status = s
        return s

    # -- backward ---------------------------------------------------------------
    def backward(self, plan: Plan, douts, stream=None):
        if plan.header_copy is not None:
            if getattr(self, "_pending", None) is plan:
                self._pending = None
            self._verify(plan)
        st = torch.cuda.current_stream(self.device).cuda_stream if stream is None else stream
        douts = [d.float().contiguous() for d in douts]
        dptr = (C.c_void_p * len(douts))(*[d.data_ptr() for d in douts])
        grads = []
        gc = (_lib.render_grads * len(plan.scenes))()
        for i, s in enumerate(plan.scenes):
            dv = torch.empty_like(s.verts)
            ds = torch.empty_like(s.sdf)
            dc = torch.empty_like(s.colors)
            gc[i].dverts, gc[i].dsdf, gc[i].dcolors = dv.data_ptr(), ds.data_ptr(), dc.data_ptr()
            grads.append((dv, ds, dc))
        check(_lib.lib().render_backward(C.byref(plan.scene_c), len(plan.scenes), C.byref(plan.view_c),
                                         len(plan.view_c), C.byref(plan.params_c), plan.kept_cap, plan.entry_cap,
                                         plan.workspace.data_ptr(), plan.workspace.numel(), dptr, C.byref(gc), st))
        plan.keep.append(douts)
        return grads

    # -- inspection -------------------------------------------------------------
    def debug(self, plan: Plan) -> dict:
        """Copies of the tiling state of a finished forward (for tests)."""
        d = _lib.render_debug_view()
        check(_lib.lib().render_debug_pointers(C.byref(plan.scene_c), len(plan.scenes), C.byref(plan.view_c),
                                               len(plan.view_c), C.byref(plan.params_c), plan.kept_cap,
                                               plan.entry_cap, plan.workspace.data_ptr(), C.byref(d)))
        stt = plan.status or self.read_status(plan)
        base = plan.workspace.data_ptr()
        ws = plan.workspace

        def grab(ptr, n, dtype):
            off = ptr - base
            nbytes = n * np.dtype(dtype).itemsize
            return ws[off:off + nbytes].cpu().numpy().view(dtype).copy()

        E = int(stt.entries)
        return dict(
            tile_keys=grab(d.tile_keys, E, np.uint32),
            entry_record=grab(d.entry_record, E, np.int32),
            kept_tet=grab(d.kept_tet, int(stt.kept), np.int32),
            view_rec_base=grab(d.view_rec_base, len(plan.view_c), np.int32),
            scene_kept_base=grab(d.scene_kept_base, len(plan.scenes), np.int32),
            scene_kept_count=grab(d.scene_kept_count, len(plan.scenes), np.int32),
            ranges=grab(d.ranges, 2 * int(d.total_tiles), np.uint32).reshape(-1, 2),
            last=grab(d.last, int(d.total_pixels), np.int32) if d.last else None,
            t_last=grab(d.t_last, int(d.total_pixels), np.float32) if d.t_last else None,
            entries=E, kept=int(stt.kept), records=int(stt.records),
        )


class TetSplatFunction(torch.autograd.Function):
    """out[B,8,H,W] = render(verts, sdf, colors; tets, cams).  Backward returns
    gradients for verts, sdf and colors."""

    @staticmethod
    def forward(ctx, verts, sdf, colors, tets, cams, s, renderer):
        scene = SceneT(verts.detach().contiguous(), tets.contiguous(), sdf.detach().contiguous(),
                       colors.detach().contiguous(), float(s))
        plan = renderer.forward([scene], cams)
        ctx.plan = plan
        ctx.renderer = renderer
        if plan.stacked is None:
            raise ValueError("TetSplatFunction renders views of one size; use Renderer for mixed sizes")
        return plan.stacked

    @staticmethod
    def backward(ctx, dout):
        dout = dout.contiguous()
        (dv, ds, dc), = ctx.renderer.backward(ctx.plan, [dout[v] for v in range(dout.shape[0])])
        ctx.plan = None
        return dv, ds, dc, None, None, None, None


def render(verts, sdf, colors, tets, cams, s, renderer: Renderer | None = None):
    """Differentiable render of one scene into [n_views, 8, H, W] (all views the
    same size).  Channels: R, G, B, opacity, depth, Nx, Ny, Nz."""
    return TetSplatFunction.apply(verts, sdf, colors, tets, np.asarray(cams, np.float32), s,
                                  renderer or Renderer())
