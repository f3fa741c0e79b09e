"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle

IMG_TOL = 1e-5     # max-abs image error vs the float32 oracle
# Gradients: "within 1e-4 relative" of the float32 oracle, read normwise per
# output, max|g - r| / max|r|.  Element-wise, |g - r| / (|r| + 1e-3 max|r|)
# against the float64 oracle, an FP32 implementation cannot do better than
# the float32 oracle itself does (cancelling per-pixel terms of the position
# and SDF gradients leave it up to ~1e-3 off); the GPU must stay within twice
# the float32 oracle's own element-wise error plus 1e-4 (the GPU sums each
# vertex's contributions in another, atomic, order than the float32 oracle).
GRAD_TOL = 1e-4


def oracle_params(P, s):
    return oracle.params_array(s, tile_w=P.tile_w, tile_h=P.tile_h, alpha_min=P.alpha_min,
                               alpha_clamp=P.alpha_clamp, t_min=P.t_min, prefilter_tf=P.prefilter_tf,
                               window=getattr(P, "window", 0))


def gpu_forward(scene, cams, P, renderer=None, device="cuda"):
    import torch
    from paper_2406_01579_amd import Renderer, SceneT
    r = renderer or Renderer(P, device=device)
    st = SceneT.from_numpy(scene, device)
    plan = r.forward([st], cams)
    torch.cuda.synchronize()
    return r, plan, [o.cpu().numpy() for o in plan.outs]


def grad_err(g, r):
    """Element-wise |g - r| / (|r| + 1e-3 max|r|)."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    den = np.abs(r) + 1e-3 * max(np.abs(r).max(), 1e-30)
    return float((np.abs(g - r) / den).max())


def grad_err_norm(g, r):
    """Normwise max|g - r| / max|r|."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-30))


def check_gradient(name, got, r32, r64, label=""):
    """Assert the gradient bar and print the errors vs both oracles."""
    got = np.asarray(got, np.float64)
    n32 = grad_err_norm(got, r32)
    e64 = grad_err(got, r64)
    o64 = grad_err(r32, r64)
    print(f"{label} {name}: normwise vs f32 {n32:.2e}; element-wise vs f64 {e64:.2e} "
          f"(f32 oracle vs f64 {o64:.2e}); element-wise vs f32 {grad_err(got, r32):.2e}")
    assert n32 <= GRAD_TOL, (name, n32)
    assert e64 <= 2.0 * o64 + GRAD_TOL, (name, e64, o64)


def near_threshold_pixels(g, cams, params, pix, s):
    """Pixels whose float64 blend takes an alpha_min, alpha_clamp or t_min
    decision within 1e-6 (relative) of the threshold: float32
    implementations may legitimately decide them differently."""
    amin, aclamp, tmin = float(params[2]), float(params[3]), float(params[4])
    out = []
    for (v, i, j) in pix:
        tr = oracle.pixel_trace(g, cams, params, int(v), int(i), int(j), prec=64)
        near = False
        for a, T in zip(tr["alpha_raw"], tr["T"]):
            if amin > 0 and abs(a - amin) <= 1e-6 * amin:
                near = True
            if abs(a - aclamp) <= 1e-6:
                near = True
            if tmin > 0 and abs(T * (1 - min(a, aclamp)) - tmin) <= 1e-6 * tmin:
                near = True
        # the tet that stopped the walk is not in the trace: test the next hit
        out.append(near)
    return np.array(out, bool)


def compare_images(imgs, g, cams, params, s, prec_ref=32, pix=None):
    """Max-abs error over all (or the listed) pixels, after excluding pixels
    with a threshold decision within rounding.  Returns (err, n_excluded, n)."""
    if pix is None:
        pix = oracle.all_pixels(cams)
    ref = oracle.render(g, cams, params, pix, prec=prec_ref)
    got = np.stack([imgs[v][:, j, i] for (v, i, j) in pix], 0)
    err = np.abs(got - ref).max(axis=1)
    bad = err > IMG_TOL
    n_ex = 0
    if bad.any():
        near = near_threshold_pixels(g, cams, params, pix[bad], s)
        n_ex = int(near.sum())
        keep = np.ones(len(pix), bool)
        keep[np.nonzero(bad)[0][near]] = False
        err = err[keep]
    return float(err.max()) if err.size else 0.0, n_ex, len(pix)


def gpu_tiling(renderer, plan):
    """GPU tiling state mapped to tet ids: (kept tet ids, sorted tile keys,
    sorted tet ids, ranges)."""
    d = renderer.debug(plan)
    nv = len(plan.view_c)
    vscene = [plan.view_c[v].scene for v in range(nv)]
    rec = d["entry_record"].astype(np.int64)
    view_of = np.zeros(rec.shape[0], np.int64)
    for v in range(nv):
        view_of[rec >= d["view_rec_base"][v]] = v
    slot = np.array([d["scene_kept_base"][vscene[v]] for v in view_of]) + rec - d["view_rec_base"][view_of]
    tets = d["kept_tet"][slot] if rec.size else np.zeros(0, np.int32)
    return d, tets
