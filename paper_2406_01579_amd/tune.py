"""Autotuner for the compositing launch shape.

The knobs are the screen tile (8x8, 16x8, 8x16, 16x16, 32x8) and, for 8x8
tiles, the per-lane work and the LDS chunk lengths.  The per-lane work is set
by the number of 64-lane waves that share a tile (1, 2, 4, 8): the waves
split a chunk's (entry, pixel) pairs between them, so one wave evaluates
eight times the pairs per lane of eight waves.  With several waves, the
entries staged in LDS per step of a tile's walk are 32 or 64 (forward) and
16 or 32 (backward): shorter chunks mean less LDS per workgroup (more of them
per CU) but more steps, each a round of barriers.  Every candidate produces
the same images and gradients (the per-pixel arithmetic and blend order do
not depend on the launch shape), so the choice is purely a speed decision.

The tuner times forward + backward of each candidate on the caller's actual
scenes and views (median of a few repetitions, HIP events on the rendering
stream) and caches the winner under a signature of the workload: the bit
lengths of the tet count and of the kept count, the image sizes, the number
of views and the steepness bucket.  The cache is a JSON file.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict

import numpy as np

from .frontend import Params

TILES = [(8, 8), (16, 8), (8, 16), (16, 16), (32, 8)]
WAVES = [1, 2, 4, 8]
CHUNKS_FWD = [32, 64]
CHUNKS_BWD = [16, 32]


def candidates():
    """(tile_w, tile_h, waves, chunk_fwd, chunk_bwd); chunk 0: the kernel's
    fixed length (the one-wave and larger-tile kernels have no chunk knob)."""
    out = []
    for tw, th in TILES:
        if (tw, th) == (8, 8):
            for w in WAVES:
                if w == 1:
                    out.append((tw, th, w, 0, 0))
                else:
                    out += [(tw, th, w, cf, cb) for cf in CHUNKS_FWD for cb in CHUNKS_BWD]
        else:
            out.append((tw, th, 1, 0, 0))
    return out


def label(cand) -> str:
    tw, th, w, cf, cb = cand
    return f"{tw}x{th}w{w}" + (f"f{cf}b{cb}" if cf else "")


def _bits(x: int) -> int:
    return int(x).bit_length()


def signature(n_tets: int, n_kept: int, sizes, n_views: int, s: float) -> str:
    """Workload bucket: tet and kept counts by bit length, distinct image
    sizes, view count, steepness by bit length."""
    sz = sorted({(int(w), int(h)) for w, h in sizes})
    return json.dumps({"tets": _bits(n_tets), "kept": _bits(n_kept), "sizes": sz, "views": n_views,
                       "s": _bits(int(round(s)))}, sort_keys=True)


class Autotuner:
    def __init__(self, cache_path: str | None = None, reps: int = 3, base: Params | None = None,
                 timer=None):
        self.cache_path = cache_path
        self.reps = reps
        self.base = base or Params()
        self.cache = {}
        self._timer = timer
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def params_for(self, cand) -> Params:
        d = asdict(self.base)
        d.update(tile_w=cand[0], tile_h=cand[1], waves=cand[2], chunk_fwd=cand[3], chunk_bwd=cand[4])
        return Params(**d)

    def tune(self, key: str, measure) -> Params:
        """measure(params) -> seconds.  Returns (and caches) the fastest."""
        if key in self.cache and len(self.cache[key].get("best", ())) == 5:   # (older entries: re-tuned)
            return self.params_for(tuple(self.cache[key]["best"]))
        times = {}
        for cand in candidates():
            t = measure(self.params_for(cand))
            times[cand] = t
        best = min(times, key=times.get)
        self.cache[key] = {"best": list(best), "ms": {label(c): round(1e3 * t, 4) for c, t in times.items()}}
        self._save()
        return self.params_for(best)

    # ------------------------------------------------------------------
    def best(self, scenes, cams, view_scene=None, dout=None, device="cuda") -> Params:
        """Tune forward + backward for these device scenes and cameras."""
        import torch

        from .frontend import Renderer
        cams = np.asarray(cams, np.float32)
        nv = cams.shape[0]
        if view_scene is None:
            view_scene = np.zeros(nv, np.int32)
        probe = Renderer(self.base, device=device, check="sync")
        plan = probe.forward(scenes, cams, view_scene)
        kept = int(plan.status.kept)
        del plan
        key = signature(sum(int(s.tets.shape[0]) for s in scenes), kept, [(c[0], c[1]) for c in cams], nv,
                        max(float(s.s) for s in scenes))
        douts = None

        def measure(params):
            nonlocal douts
            # the first call sizes the workspace synchronously, the timed ones
            # check their status without waiting
            r = Renderer(params, device=device, check="lazy")
            if douts is None:
                p0 = r.forward(scenes, cams, view_scene)
                douts = [torch.randn_like(o) for o in p0.outs] if dout is None else dout
                del p0
            ts = []
            for k in range(self.reps + 1):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                p = r.forward(scenes, cams, view_scene)
                r.backward(p, douts)
                b.record()
                torch.cuda.synchronize()
                if k > 0:
                    ts.append(a.elapsed_time(b) * 1e-3)
            return float(np.median(ts))

        return self.tune(key, self._timer or measure)
