"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle

IMG_TOL = 1e-5     # max-abs image error vs the float32 oracle
# Gradients, two bars.
# 1. "Within 1e-4 relative" of the float32 oracle, read normwise per output:
#    max|g - r32| / max|r32| <= 1e-4.
# 2. Element-wise against the float64 oracle, a bound derived per element from
#    the oracle's error budget (oracle.backward_budget):
#        |g - r64| <= 2 E + gamma_{N + 32} A,   gamma_n = n u / (1 - n u), u = 2^-24.
#    Every element is a sum of N per-(pixel, tet) terms carried to the vertex
#    by a linear chain J.  E is the float32 oracle's own error in those terms,
#    summed in absolute value; the kernels evaluate the same terms in float32
#    with another exponential, reciprocal and operation order and are allowed
#    twice that.  gamma_{N + 32} A bounds any order and grouping of the float32
#    sums (N terms; 32 covers the float32 chain through the projection, the
#    mean depth and the normal) carried through |J|.  An element no term
#    reaches must be exactly zero.
GRAD_TOL = 1e-4
U32 = 2.0 ** -24
CHAIN_OPS = 32


def gamma(n):
    n = np.asarray(n, np.float64)
    return n * U32 / (1.0 - n * U32)


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


def grad_err_norm(g, r):
    """Normwise max|g - r| / max|r|."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-30))


def grad_bound(A, E, N):
    """Element-wise bound on a float32 gradient's distance to the float64 oracle."""
    return 2.0 * E + gamma(N + CHAIN_OPS) * A


def check_gradient(name, got, r32, r64, label, budget):
    """Assert both gradient bars and print the errors vs both oracles."""
    got = np.asarray(got, np.float64)
    A, E, N = budget
    bound = grad_bound(A, E, N)
    err = np.abs(got - r64)
    n32 = grad_err_norm(got, r32)
    reach = bound > 0
    ratio = float((err[reach] / bound[reach]).max()) if reach.any() else 0.0
    own = float((np.abs(r32 - r64)[reach] / bound[reach]).max()) if reach.any() else 0.0
    print(f"{label} {name}: normwise vs f32 {n32:.2e}; vs f64 {grad_err_norm(got, r64):.2e} normwise, "
          f"{ratio:.3f} of the element bound (f32 oracle {own:.3f}); f32 oracle vs f64 "
          f"{grad_err_norm(r32, r64):.2e} normwise")
    assert n32 <= GRAD_TOL, (name, n32)
    assert np.all(got[~reach] == 0.0), (name, "gradient on an element no term reaches")
    assert ratio <= 1.0, (name, ratio)


def oracle_gradients(g, cams, params, pix, dflat):
    """Float32 and float64 oracle gradients and the float32 error budget."""
    r32 = oracle.backward(g, cams, params, pix, dflat, prec=32)
    r64 = oracle.backward(g, cams, params, pix, dflat, prec=64)
    b = oracle.backward_budget(g, cams, params, pix, dflat)
    return r32, r64, b


def check_gradients(got, refs, label):
    """got: (dverts, dsdf, dcolors) tensors or arrays; refs from oracle_gradients."""
    r32, r64, b = refs
    for k, name in enumerate(("dverts", "dsdf", "dcolors")):
        x = got[k]
        x = x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)
        check_gradient(name, x, r32[k], r64[k], label, (b["A"][k], b["E"][k], b["N"][k]))


def near_threshold_pixels(g, cams, params, pix, s):
    """Pixels whose walk takes a skip (alpha_min), clamp (alpha_clamp) or stop
    (t_min) decision closer to its threshold than twice the running error
    bound of the quantity decided on: float32 implementations may take it
    either way.  Every candidate's decisions count, the stopping one's too."""
    out = []
    for (v, i, j) in pix:
        d = oracle.pixel_decisions(g, cams, params, int(v), int(i), int(j))
        active = ((d["kind"] == 0) & (d["threshold"] > 0)) | ((d["kind"] == 1) & (d["threshold"] < 1)) | \
                 ((d["kind"] == 2) & (d["threshold"] > 0))
        near = np.abs(d["value"] - d["threshold"]) <= 2.0 * d["bound"]
        out.append(bool(np.any(active & near)))
    return np.array(out, bool)


def compare_images(imgs, g, cams, params, s, prec_ref=32, pix=None):
    """Max-abs error over all (or the listed) pixels vs the float32 oracle.

    A pixel over IMG_TOL is excluded (and counted) when either
    - its walk takes a threshold decision within rounding of the threshold
      (near_threshold_pixels: float32 implementations may decide it either
      way), or
    - in every channel over IMG_TOL the kernels' value is at least as close to
      the float64 oracle as the float32 oracle's is: the miss is the float32
      oracle's own rounding.
    Returns (err, n_excluded, n)."""
    if pix is None:
        pix = oracle.all_pixels(cams)
    ref = oracle.render(g, cams, params, pix, prec=prec_ref)
    got = np.stack([imgs[v][:, j, i] for (v, i, j) in pix], 0)
    err = np.abs(got - ref).max(axis=1)
    bad = np.nonzero(err > IMG_TOL)[0]
    n_ex = 0
    if bad.size:
        near = near_threshold_pixels(g, cams, params, pix[bad], s)
        r64 = oracle.render(g, cams, params, pix[bad], prec=64)
        over = np.abs(got[bad] - ref[bad]) > IMG_TOL
        own = np.all(~over | (np.abs(got[bad] - r64) <= np.abs(ref[bad] - r64)), axis=1)
        excl = near | own
        for q in range(bad.size):
            print(f"  pixel {tuple(int(x) for x in pix[bad[q]])}: {err[bad[q]]:.3e} vs f32, "
                  f"{np.abs(got[bad[q]] - r64[q]).max():.3e} vs f64 (f32 oracle "
                  f"{np.abs(ref[bad[q]] - r64[q]).max():.3e}); near a threshold {bool(near[q])}")
        n_ex = int(excl.sum())
        keep = np.ones(len(pix), bool)
        keep[bad[excl]] = False
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
