"""Forward-only serving loop over resident scenes.

Scenes are uploaded once into a registry and stay resident in HBM.  A
request names a scene and carries 1..n cameras (any image sizes); its result
is one [8, H, W] image per camera.  The scheduler admits a request when its
HBM footprint (workspace + outputs, computed from the library's own
workspace sizing) fits the free part of the budget, and batches continuously:
whenever one of the executor's streams is idle, every queued request that
fits (FIFO, up to a view and pixel limit) goes into ONE multi-scene launch
of the rasterizer on that stream, while the other streams' launches still
run.  Capacities come from per-scene probes; a launch that outgrows them is
detected from its status header (copied to pinned memory on the stream, no
host wait) and re-run with the exact sizes before its requests complete, so
no request ever receives an image from an overflowed launch.

Latency is arrival -> completion, where completion is the device timestamp
of the event recorded after the request's launch (plus re-runs), placed on
the host clock through a reference event recorded when the server clock
starts.

The plain path for comparison (``batching=False, streams=1``) serves the same
trace FIFO with one launch sequence per view.
"""
from __future__ import annotations

import ctypes as C
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import check
from .frontend import Params, Renderer, SceneT

OUT_CHANNELS = 8


# ----------------------------------------------------------------------------
# requests and the host-side scheduling policy (no GPU work)
# ----------------------------------------------------------------------------
@dataclass
class Request:
    id: int
    scene: int
    cams: np.ndarray                  # [nv, 22] float32 camera rows
    arrival: float                    # seconds on the server clock
    footprint: int = 0                # bytes while in flight
    outs: list | None = None          # [8, H, W] device tensors, one per camera
    done_at: float | None = None      # seconds on the server clock
    error: str | None = None
    batch: int = -1

    @property
    def views(self) -> int:
        return int(self.cams.shape[0])

    @property
    def pixels(self) -> int:
        return int(sum(int(c[0]) * int(c[1]) for c in self.cams))

    def done(self) -> bool:
        return self.done_at is not None or self.error is not None

    @property
    def latency(self) -> float:
        return self.done_at - self.arrival


class Scheduler:
    """Admission by HBM footprint and FIFO batch formation.

    ``submit`` rejects a request whose footprint alone exceeds the budget and
    queues the rest.  ``next_batch`` takes queued requests from the head while
    the batch stays within ``max_views`` / ``max_pixels`` and the in-flight
    bytes stay within the budget; it stops at the first request that does not
    fit, so no request is overtaken.  Without batching a batch is one
    request."""

    def __init__(self, budget_bytes: int, max_views: int = 32, max_pixels: int = 16 << 20,
                 batching: bool = True):
        self.budget = int(budget_bytes)
        self.max_views = max_views
        self.max_pixels = max_pixels
        self.batching = batching
        self.queue: deque = deque()
        self.in_flight = 0
        self.max_in_flight = 0
        self.max_queue = 0
        self.rejected = 0

    def submit(self, req: Request) -> bool:
        if req.footprint > self.budget:
            req.error = f"request needs {req.footprint} bytes, over the {self.budget}-byte budget"
            self.rejected += 1
            return False
        self.queue.append(req)
        self.max_queue = max(self.max_queue, len(self.queue))
        return True

    def next_batch(self) -> list:
        batch, views, pixels, nbytes = [], 0, 0, 0
        while self.queue:
            r = self.queue[0]
            if batch and (not self.batching or views + r.views > self.max_views
                          or pixels + r.pixels > self.max_pixels):
                break
            if self.in_flight + nbytes + r.footprint > self.budget:
                break
            batch.append(self.queue.popleft())
            views += r.views
            pixels += r.pixels
            nbytes += r.footprint
        self.in_flight += nbytes
        self.max_in_flight = max(self.max_in_flight, self.in_flight)
        return batch

    def charge(self, nbytes: int):
        """Bytes beyond the admitted footprints that a running launch took
        (a re-run with larger capacities); released with its batch."""
        self.in_flight += int(nbytes)
        self.max_in_flight = max(self.max_in_flight, self.in_flight)

    def release(self, batch, extra: int = 0):
        self.in_flight -= sum(r.footprint for r in batch) + int(extra)


# ----------------------------------------------------------------------------
# resident scenes
# ----------------------------------------------------------------------------
class SceneRegistry:
    """Scenes resident in HBM with their sizing data: the number of tets the
    pre-filter keeps (view-independent) and, per probed image size, the
    (tet, tile) entries one view produces."""

    def __init__(self, params: Params | None = None, device="cuda", margin: float = 1.5):
        self.params = params or Params()
        self.device = torch.device(device)
        self.margin = margin
        self.scenes: list[SceneT] = []
        self.kept: list[int] = []
        self.entries: list[dict] = []     # per scene: {(W, H): entries per view}
        self.bytes = 0

    def add(self, scene, probe_cams) -> int:
        """Upload a scene (numpy arrays or SceneT) and probe its sizing with
        the given cameras (one synchronous launch per distinct image size)."""
        sc = scene if isinstance(scene, SceneT) else SceneT.from_numpy(scene, self.device)
        probe = Renderer(self.params, device=self.device, check="sync")
        probe_cams = np.asarray(probe_cams, np.float32)
        per_size, kept = {}, 0
        for size in sorted({(int(c[0]), int(c[1])) for c in probe_cams}):
            cams = probe_cams[[(int(c[0]), int(c[1])) == size for c in probe_cams]]
            plan = probe.forward([sc], cams)
            per_size[size] = int(plan.status.entries_needed) / len(cams)
            kept = int(plan.status.kept)
            del plan
        self.scenes.append(sc)
        self.kept.append(kept)
        self.entries.append(per_size)
        self.bytes += sum(t.numel() * t.element_size() for t in (sc.verts, sc.tets, sc.sdf, sc.colors))
        return len(self.scenes) - 1

    def est_entries(self, sid: int, W: int, H: int) -> int:
        table = self.entries[sid]
        if (W, H) in table:
            e = table[(W, H)]
        else:
            # nearest probed size by pixel count, scaled up (never down) by the pixel ratio
            (pw, ph), e = min(table.items(), key=lambda kv: abs(kv[0][0] * kv[0][1] - W * H))
            e *= max(1.0, (W * H) / (pw * ph))
        return int(e * self.margin) + 256

    def grow(self, sid: int, W: int, H: int, factor: float):
        table = self.entries[sid]
        table[(W, H)] = max(table.get((W, H), 0.0), self.est_entries(sid, W, H) / self.margin) * factor


# ----------------------------------------------------------------------------
# executor
# ----------------------------------------------------------------------------
@dataclass
class _Launch:
    requests: list
    plans: list = field(default_factory=list)
    args: list = field(default_factory=list)   # per plan: (scenes, cams, view_scene, caps)
    headers: list = field(default_factory=list)
    end: object = None
    reruns: int = 0
    extra_bytes: int = 0   # workspace its re-runs took beyond the admitted footprints


class Server:
    def __init__(self, registry: SceneRegistry, streams: int = 2, budget_bytes: int | None = None,
                 max_views: int = 32, max_pixels: int = 16 << 20, batching: bool = True,
                 keep_outputs: bool = True):
        self.reg = registry
        self.keep_outputs = keep_outputs
        self.device = registry.device
        self.renderer = Renderer(registry.params, device=self.device, check="none")
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(0.5 * free)
        self.sched = Scheduler(budget_bytes, max_views, max_pixels, batching)
        self.batching = batching
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, streams))]
        self.slots: list = [None] * len(self.streams)
        self.requests: list[Request] = []
        self.launches = 0
        self.reruns = 0
        self.batch_views: list[int] = []
        self._start_clock()

    # -- clock ---------------------------------------------------------------
    def _start_clock(self):
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref.record(torch.cuda.current_stream(self.device))
        self._ref.synchronize()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- sizing --------------------------------------------------------------
    def _caps(self, sids, cams, view_scene):
        kept = sum(self.reg.kept[s] for s in sids) + 256
        ent = sum(self.reg.est_entries(sids[int(view_scene[v])], int(cams[v][0]), int(cams[v][1]))
                  for v in range(len(cams)))
        return kept, ent + 1024

    def footprint(self, sid: int, cams) -> int:
        cams = np.asarray(cams, np.float32)
        vs = np.zeros(len(cams), np.int32)
        kept, ent = self._caps([sid], cams, vs)
        scene_c = (_lib.render_scene * 1)(self.reg.scenes[sid].c())
        view_c = (_lib.render_view * len(cams))()
        for v, c in enumerate(cams):
            view_c[v].scene, view_c[v].width, view_c[v].height = 0, int(c[0]), int(c[1])
        params_c = self.reg.params.c()
        n = C.c_size_t(0)
        check(_lib.lib().render_workspace_size(C.byref(scene_c), 1, C.byref(view_c), len(cams),
                                               C.byref(params_c), kept, ent, C.byref(n)))
        return int(n.value) + sum(4 * OUT_CHANNELS * int(c[0]) * int(c[1]) for c in cams)

    # -- requests --------------------------------------------------------------
    def submit(self, scene: int, cams, arrival: float | None = None) -> Request:
        cams = np.asarray(cams, np.float32)
        if cams.ndim == 1:
            cams = cams[None]
        if not 0 <= scene < len(self.reg.scenes):
            raise ValueError(f"unknown scene {scene}")
        r = Request(len(self.requests), scene, cams, self.now() if arrival is None else arrival)
        r.footprint = self.footprint(scene, cams)
        self.requests.append(r)
        self.sched.submit(r)
        return r

    # -- launches --------------------------------------------------------------
    def _launch_plan(self, L: _Launch, stream, sids, cams, vs, caps):
        with torch.cuda.stream(stream):
            plan = self.renderer.forward([self.reg.scenes[s] for s in sids], cams, vs, caps=caps)
            hdr = torch.empty(_lib.STATUS_BYTES, dtype=torch.uint8, pin_memory=True)
            hdr.copy_(plan.workspace[:_lib.STATUS_BYTES], non_blocking=True)
        L.plans.append(plan)
        L.headers.append(hdr)
        L.args.append((sids, cams, vs, caps))
        self.launches += 1

    def _start(self, k: int, batch: list):
        L = _Launch(batch)
        st = self.streams[k]
        if self.batching:
            sids, cams, vs = [], [], []
            for r in batch:
                if r.scene not in sids:
                    sids.append(r.scene)
                cams.append(r.cams)
                vs += [sids.index(r.scene)] * r.views
            cams = np.concatenate(cams, 0)
            vs = np.asarray(vs, np.int32)
            self._launch_plan(L, st, sids, cams, vs, self._caps(sids, cams, vs))
        else:
            for r in batch:
                for v in range(r.views):
                    cams = r.cams[v:v + 1]
                    vs = np.zeros(1, np.int32)
                    self._launch_plan(L, st, [r.scene], cams, vs, self._caps([r.scene], cams, vs))
        L.end = torch.cuda.Event(enable_timing=True)
        L.end.record(st)
        self.batch_views.append(sum(r.views for r in batch))
        for r in batch:
            r.batch = len(self.batch_views) - 1
        self.slots[k] = L

    def _finish(self, k: int) -> int:
        L = self.slots[k]
        st = self.streams[k]
        redo = False
        for i, hdr in enumerate(L.headers):
            s = _lib.render_status()
            check(_lib.lib().render_decode_status(hdr.data_ptr(), C.byref(s)))
            if s.invalid_index:
                for r in L.requests:
                    r.error = "a tet of the scene has a vertex index outside [0, V)"
            if s.overflow & 3:   # (bit 2 concerns a backward only: a served forward stands)
                # outgrown capacities: re-run this launch with the exact sizes and
                # remember larger estimates for the scene/size pairs it holds
                sids, cams, vs, caps = L.args[i]
                need = (int(s.kept) + 256, int(int(s.entries_needed) * 1.05) + 1024)
                factor = max(1.0, need[1] / max(1, caps[1])) * 1.25
                # once per (scene, image size) of the launch, not once per view
                for sid, W, H in sorted({(sids[int(vs[v])], int(cams[v][0]), int(cams[v][1]))
                                         for v in range(len(cams))}):
                    self.reg.grow(sid, W, H, factor)
                old_bytes = L.plans[i].workspace.numel()
                with torch.cuda.stream(st):
                    plan = self.renderer.forward([self.reg.scenes[x] for x in sids], cams, vs, caps=need)
                    hdr2 = torch.empty(_lib.STATUS_BYTES, dtype=torch.uint8, pin_memory=True)
                    hdr2.copy_(plan.workspace[:_lib.STATUS_BYTES], non_blocking=True)
                # the larger workspace counts against the HBM budget until the batch completes
                grown = max(0, plan.workspace.numel() - old_bytes)
                L.extra_bytes += grown
                self.sched.charge(grown)
                L.plans[i], L.headers[i], L.args[i] = plan, hdr2, (sids, cams, vs, need)
                L.reruns += 1
                self.reruns += 1
                self.launches += 1
                redo = True
        if redo:
            L.end = torch.cuda.Event(enable_timing=True)
            L.end.record(st)
            return 0
        t_done = self._ref.elapsed_time(L.end) * 1e-3
        outs = [o for p in L.plans for o in p.outs]
        j = 0
        for r in L.requests:
            r.outs = outs[j:j + r.views] if self.keep_outputs else None
            j += r.views
            if r.error is None:
                r.done_at = t_done
        self.sched.release(L.requests, L.extra_bytes)
        self.slots[k] = None
        return len(L.requests)

    def poll(self) -> int:
        """Complete finished launches and start new ones on idle streams.
        Returns the number of requests completed."""
        done = 0
        for k, L in enumerate(self.slots):
            if L is not None and L.end.query():
                done += self._finish(k)
        for k, L in enumerate(self.slots):
            if L is None and self.sched.queue:
                batch = self.sched.next_batch()
                if not batch:
                    break
                self._start(k, batch)
        return done

    def busy(self) -> bool:
        return bool(self.sched.queue) or any(L is not None for L in self.slots)

    def drain(self):
        while self.busy():
            if self.poll() == 0:
                time.sleep(20e-6)

    # -- open-loop trace -----------------------------------------------------
    def run(self, trace) -> dict:
        """Serve an open-loop trace [(arrival_s, scene, cams), ...] in real
        time (arrivals relative to now) and return the statistics."""
        self._start_clock()
        first = len(self.requests)
        i, n = 0, len(trace)
        while i < n or self.busy():
            now = self.now()
            while i < n and trace[i][0] <= now:
                self.submit(trace[i][1], trace[i][2], arrival=trace[i][0])
                i += 1
            if self.poll() == 0:
                if not self.busy() and i < n:
                    time.sleep(max(0.0, min(trace[i][0] - self.now(), 1e-3)))
                else:
                    time.sleep(20e-6)
        return self.stats(self.requests[first:])

    def stats(self, reqs) -> dict:
        ok = [r for r in reqs if r.done_at is not None]
        lat = np.array([r.latency for r in ok]) * 1e3
        span = max(r.done_at for r in ok) - min(r.arrival for r in ok) if ok else 0.0
        px = sum(r.pixels for r in ok)
        return {
            "requests": len(reqs), "served": len(ok), "rejected": sum(r.error is not None for r in reqs),
            "p50_ms": float(np.percentile(lat, 50)) if ok else None,
            "p99_ms": float(np.percentile(lat, 99)) if ok else None,
            "mean_ms": float(lat.mean()) if ok else None,
            "mpix_per_s": px / span / 1e6 if span > 0 else None,
            "launches": self.launches, "reruns": self.reruns,
            "batches": len(self.batch_views),
            "mean_views_per_batch": float(np.mean(self.batch_views)) if self.batch_views else 0.0,
            "max_queue": self.sched.max_queue, "max_in_flight_bytes": self.sched.max_in_flight,
            "budget_bytes": self.sched.budget, "resident_scene_bytes": self.reg.bytes,
        }
