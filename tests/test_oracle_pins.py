"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the passage of the paper it checks.  The checks use closed
forms, an independent 3D ray route (tests/ref3d.py), library routines
(numpy.linalg, scipy.spatial), brute force on tiny inputs, and derivatives by
central finite differences and by forward-mode dual numbers.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
import synth
from tests import ref3d

EXACT = dict(alpha_min=0.0, alpha_clamp=1.0, t_min=0.0)


# ---------------------------------------------------------------------------
# Eq. 1 (Sec. 3.2)
# ---------------------------------------------------------------------------
def _alpha_decimal(fp, fn, s, prec=1200):
    """Eq. 1 as printed, evaluated with 1200 significant digits (enough for the cancellation when both logistic values round near 1)."""
    getcontext().prec = prec
    def phi(x):
        return Decimal(1) / (Decimal(1) + (Decimal(-s) * Decimal(x)).exp())
    pp, pn = phi(fp), phi(fn)
    return max((pp - pn) / pp, Decimal(0))


def test_eq1_closed_forms(oracle_lib):
    # f_prev = delta, f_next = -delta  ->  alpha = 1 - exp(-s delta)
    assert oracle.alpha(0.1, -0.1, 20.0) == pytest.approx(0.864664716763387, abs=1e-15)
    assert oracle.alpha(0.01, -0.01, 320.0) == pytest.approx(0.959237796021634, abs=1e-15)
    # f_prev <= f_next -> 0 (the max(., 0) of Eq. 1)
    assert oracle.alpha(-0.2, 0.3, 50.0) == 0.0
    assert oracle.alpha(0.25, 0.25, 50.0) == 0.0


def test_eq1_stable_form_equals_literal(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(400):
        s = float(rng.choice([20.0, 100.0, 320.0, 620.0, 2000.0]))
        fp, fn = rng.uniform(-0.6, 0.6, size=2)
        ref = float(_alpha_decimal(float(fp), float(fn), s))
        got = oracle.alpha(float(fp), float(fn), s)
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-300)


def test_eq1_large_s_limit(oracle_lib):
    # as s grows, alpha -> 1 when f_next < 0 < ... and f_prev > f_next, -> 0 when f_next > 0
    s = 1e4
    assert oracle.alpha(0.05, -0.05, s) == pytest.approx(1.0, abs=1e-12)   # crossing the surface
    assert oracle.alpha(0.2, 0.1, s) < 1e-100                             # outside the surface
    # both negative (behind the surface): the literal formula also tends to 1
    assert oracle.alpha(-0.1, -0.2, s) == pytest.approx(1.0, abs=1e-12)
    assert float(_alpha_decimal(-0.1, -0.2, s)) == pytest.approx(1.0, abs=1e-12)


# ---------------------------------------------------------------------------
# Pre-filter (Sec. 3.2)
# ---------------------------------------------------------------------------
def test_prefilter_bound_and_flat_tets(oracle_lib):
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    g = oracle.Geometry.of(sc)
    P = oracle.params_array(20.0, **EXACT)
    keep, amax, _, _, _ = oracle.prefilter(g, P)
    f = sc.sdf.astype(np.float64)[sc.tets]
    # alpha_max from (max, min) vertex SDF, independently evaluated
    for k in np.random.default_rng(1).choice(sc.K, 200, replace=False):
        ref = float(_alpha_decimal(f[k].max(), f[k].min(), 20.0))
        assert amax[k] == pytest.approx(ref, rel=2e-6, abs=1e-30)
        assert keep[k] == (amax[k] >= np.float32(1 / 255))
    # every blended alpha stays below its tet's bound
    for (i, j) in [(32, 32), (25, 30), (40, 28), (20, 20), (44, 40)]:
        tr = oracle.pixel_trace(g, w.cams, P, 0, i, j)
        assert len(tr["tet"]) > 0
        for k, a in zip(tr["tet"], tr["alpha_raw"]):
            assert a <= float(_alpha_decimal(f[k].max(), f[k].min(), 20.0)) * (1 + 1e-12) + 1e-15
    # a tet with constant SDF has alpha_max = 0 and is dropped
    flat = synth.Scene(sc.verts, sc.tets[:1], np.full_like(sc.sdf, -0.3), sc.colors, 20.0)
    keep1, amax1, *_ = oracle.prefilter(oracle.Geometry.of(flat), P)
    assert amax1[0] == 0.0 and not keep1[0]


def test_prefilter_does_not_change_default_output(oracle_lib):
    """With alpha_min = T_f every dropped tet would have been skipped anyway."""
    w = synth.tiny(s=20.0)
    g = oracle.Geometry.of(w.scenes[0])
    on = oracle.render_images(g, w.cams, oracle.params_array(20.0))[0]
    off = oracle.render_images(g, w.cams, oracle.params_array(20.0, prefilter_tf=0.0))[0]
    assert np.array_equal(on, off)


# ---------------------------------------------------------------------------
# Per-tet normal (Sec. 3.2, App. A.3)
# ---------------------------------------------------------------------------
def _deformed_grid(R, seed, amp=0.2):
    rng = np.random.default_rng(seed)
    v, t = synth.kuhn_grid(R)
    h = 2.0 / R
    v = v + rng.uniform(-amp * h, amp * h, size=v.shape)
    return v, t


def test_normal_of_linear_sdf(oracle_lib):
    v, t = _deformed_grid(4, 3)
    a = np.array([0.3, -1.2, 0.7])
    sdf = v @ a + 0.05
    g = oracle.Geometry(v, t, sdf, np.zeros_like(v))
    P = oracle.params_array(20.0, prefilter_tf=0.0)
    keep, _, nrm, _, grad = oracle.prefilter(g, P)
    assert keep.all()
    np.testing.assert_allclose(grad, np.broadcast_to(a, grad.shape), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(nrm, np.broadcast_to(a / np.linalg.norm(a), nrm.shape), atol=1e-12)


def test_normal_matches_edge_system_and_vertex_order(oracle_lib):
    v, t = _deformed_grid(3, 4)
    rng = np.random.default_rng(5)
    sdf = rng.normal(size=v.shape[0])
    g = oracle.Geometry(v, t, sdf, np.zeros_like(v))
    P = oracle.params_array(20.0, prefilter_tf=0.0)
    _, _, nrm, _, grad = oracle.prefilter(g, P)
    for k in range(t.shape[0]):
        E = v[t[k, 1:]] - v[t[k, 0]]
        ref = np.linalg.solve(E, sdf[t[k, 1:]] - sdf[t[k, 0]])
        np.testing.assert_allclose(grad[k], ref, rtol=1e-9, atol=1e-9)
    perm = t[:, [2, 0, 3, 1]]
    _, _, nrm2, _, _ = oracle.prefilter(oracle.Geometry(v, perm, sdf, np.zeros_like(v)), P)
    np.testing.assert_allclose(nrm2, nrm, atol=1e-12)


def test_normal_of_degenerate_tet_is_zero(oracle_lib):
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64)  # coplanar
    t = np.array([[0, 1, 2, 3]], np.int32)
    g = oracle.Geometry(v, t, np.array([0.1, -0.2, 0.3, -0.1]), np.zeros_like(v))
    _, _, nrm, _, _ = oracle.prefilter(g, oracle.params_array(20.0, prefilter_tf=0.0))
    assert np.all(nrm == 0.0)


# ---------------------------------------------------------------------------
# Barycentrics and perspective correction (App. A.1-A.2) vs the 3D ray route
# ---------------------------------------------------------------------------
def test_2d_route_equals_3d_ray_route(oracle_lib):
    rng = np.random.default_rng(11)
    cam = synth.orbit_camera(0.3, 0.2, 2.5, 50.0, 64, 64)
    Rm, tt, fx, fy, cx, cy = ref3d.cam_parts(cam)
    n_hit = 0
    for _ in range(300):
        c = rng.uniform(-0.3, 0.3, 3)
        X = c + rng.normal(scale=0.15, size=(4, 3))
        f = rng.normal(scale=0.2, size=4)
        Xc = X @ Rm.T + tt
        px = fx * Xc[:, 0] / Xc[:, 2] + cx
        py = fy * Xc[:, 1] / Xc[:, 2] + cy
        for _ in range(8):
            w = rng.dirichlet(np.ones(4))
            qx, qy = w @ px + rng.normal(scale=0.5), w @ py + rng.normal(scale=0.5)
            got = oracle.tet_pixel(px, py, Xc[:, 2], f, qx, qy, 100.0)
            ref = ref3d.ray_tet(Xc, f, ref3d.ray_dir(cam, qx, qy))
            if ref is None or got[0] == 0.0:
                # allowed to disagree only within rounding of a silhouette edge
                if (ref is None) != (got[0] == 0.0):
                    margin = ref[1] - ref[0] if ref is not None else got[4] - got[3]
                    assert abs(margin) < 1e-9
                continue
            n_hit += 1
            assert got[3] == pytest.approx(ref[0], rel=1e-12)   # entry depth
            assert got[4] == pytest.approx(ref[1], rel=1e-12)   # exit depth
            assert got[1] == pytest.approx(ref[2], abs=1e-12)   # f_prev
            assert got[2] == pytest.approx(ref[3], abs=1e-12)   # f_next
    assert n_hit > 500


def test_barycentric_at_vertex_pixel(oracle_lib):
    # a pixel centre exactly at a projected vertex sees that vertex's SDF at
    # entry and exit when the vertex is the nearest point of the tet
    px = np.array([10.5, 30.5, 20.5, 20.5])
    py = np.array([10.5, 12.5, 30.5, 18.5])
    Z = np.array([2.0, 2.2, 2.4, 1.8])
    f = np.array([0.1, -0.3, 0.2, 0.5])
    out = oracle.tet_pixel(px, py, Z, f, 20.5, 18.5, 50.0)
    assert out[0] == 1.0
    assert out[3] == pytest.approx(1.8, rel=1e-14)
    assert out[1] == pytest.approx(0.5, abs=1e-14)


# ---------------------------------------------------------------------------
# Coverage: brute force against a library convex-hull test
# ---------------------------------------------------------------------------
def test_single_tet_coverage_is_projected_hull(oracle_lib):
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(12)
    cam = synth.orbit_camera(1.1, 0.4, 2.5, 50.0, 48, 48)
    Rm, tt, fx, fy, cx, cy = ref3d.cam_parts(cam)
    for trial in range(6):
        X = rng.uniform(-0.5, 0.5, size=(4, 3))
        Xc = X @ Rm.T + tt
        sdf = -(Xc[:, 2] - Xc[:, 2].mean()) * 2.0 + 0.01  # decreasing with depth -> alpha > 0 inside
        g = oracle.Geometry(X, np.array([[0, 1, 2, 3]], np.int32), sdf, np.ones((4, 3)) * 0.5)
        P = oracle.params_array(30.0, prefilter_tf=0.0, **EXACT)
        img = oracle.render_images(g, cam[None], P)[0]
        px = fx * Xc[:, 0] / Xc[:, 2] + cx
        py = fy * Xc[:, 1] / Xc[:, 2] + cy
        jj, ii = np.meshgrid(np.arange(48) + 0.5, np.arange(48) + 0.5, indexing="ij")
        q = np.stack([ii.ravel(), jj.ravel()], 1)
        inside = Delaunay(np.stack([px, py], 1)).find_simplex(q) >= 0
        # distance of each centre to the hull boundary, to skip exact ties
        hull = Delaunay(np.stack([px, py], 1)).convex_hull
        P2 = np.stack([px, py], 1)
        dmin = np.full(q.shape[0], np.inf)
        for a, b in hull:
            e = P2[b] - P2[a]
            tpar = np.clip(((q - P2[a]) @ e) / (e @ e), 0, 1)
            dmin = np.minimum(dmin, np.linalg.norm(q - (P2[a] + tpar[:, None] * e), axis=1))
        covered = img[3].ravel() > 0
        ok = dmin > 1e-6
        assert np.array_equal(covered[ok], inside[ok]), trial
        assert inside.sum() > 5


# ---------------------------------------------------------------------------
# Compositing (Eq. 2)
# ---------------------------------------------------------------------------
def test_two_tets_closed_form(oracle_lib):
    """Two tets on the optical axis, one behind the other."""
    cam = synth.orbit_camera(0.0, 0.0, 2.5, 50.0, 32, 32, bg=(0.2, 0.4, 0.6))
    Rm, tt, fx, fy, cx, cy = ref3d.cam_parts(cam)
    base = np.array([[-0.2, -0.2, -0.2], [0.3, -0.1, 0.05], [-0.1, 0.35, 0.0], [0.05, 0.0, 0.3]])
    # camera looks along -x from +x: push the second tet further along -x
    X = np.concatenate([base + [0.4, 0.0, 0.0], base + [-0.5, 0.02, 0.01]], 0)
    tets = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    Xc = X @ Rm.T + tt
    sdf = np.concatenate([0.3 - 0.4 * (Xc[:4, 2] - 2.0), 0.1 - 0.6 * (Xc[4:, 2] - 2.0)])
    col = np.random.default_rng(2).uniform(size=(8, 3))
    g = oracle.Geometry(X, tets, sdf, col)
    P = oracle.params_array(15.0, prefilter_tf=0.0, **EXACT)
    img = oracle.render_images(g, cam[None], P)[0]
    bg = np.array([0.2, 0.4, 0.6])
    n_both = 0
    for (i, j) in [(16, 16), (15, 17), (17, 15), (14, 14), (18, 18)]:
        d = ref3d.ray_dir(cam, i + 0.5, j + 0.5)
        h1 = ref3d.ray_tet(Xc[:4], sdf[:4], d)
        h2 = ref3d.ray_tet(Xc[4:], sdf[4:], d)
        a1 = ref3d.alpha_literal(h1[2], h1[3], 15.0) if h1 else 0.0
        a2 = ref3d.alpha_literal(h2[2], h2[3], 15.0) if h2 else 0.0
        c1, c2 = col[:4].mean(0), col[4:].mean(0)
        z1, z2 = Xc[:4, 2].mean(), Xc[4:, 2].mean()
        assert z1 < z2
        C = a1 * c1 + (1 - a1) * a2 * c2 + (1 - a1) * (1 - a2) * bg
        np.testing.assert_allclose(img[0:3, j, i], C, atol=1e-12)
        assert img[3, j, i] == pytest.approx(a1 + (1 - a1) * a2, abs=1e-12)
        assert img[4, j, i] == pytest.approx(a1 * z1 + (1 - a1) * a2 * z2, abs=1e-12)
        n_both += (a1 > 0.01) and (a2 > 0.01)
    assert n_both >= 3


def test_empty_scene_gives_background(oracle_lib):
    w = synth.tiny(s=20.0, bg=(0.25, 0.5, 0.75))
    sc = w.scenes[0]
    g = oracle.Geometry(sc.verts, sc.tets, np.full(sc.V, 2.0), sc.colors)  # far outside: all dropped
    P = oracle.params_array(20.0)
    img = oracle.render_images(g, w.cams, P)[0]
    np.testing.assert_array_equal(img[0:3], np.broadcast_to(np.array([0.25, 0.5, 0.75])[:, None, None], img[0:3].shape))
    assert np.all(img[3:] == 0)
    pix = oracle.all_pixels(w.cams)
    dv, ds, dc = oracle.backward(g, w.cams, P, pix, np.ones((pix.shape[0], 8)))
    assert np.all(dv == 0) and np.all(ds == 0) and np.all(dc == 0)


def test_transmittance_and_opacity_identities(oracle_lib):
    w = synth.tiny(s=100.0)
    g = oracle.Geometry.of(w.scenes[0])
    for P in (oracle.params_array(100.0), oracle.params_array(100.0, **EXACT)):
        out, nb, tf = oracle.render(g, w.cams, P, want_state=True)
        assert np.all(out[:, 3] >= 0) and np.all(out[:, 3] <= 1 + 1e-12)
        np.testing.assert_allclose(out[:, 3], 1 - tf, atol=1e-12)   # sum T a = 1 - prod(1-a)
        for (i, j) in [(32, 32), (30, 22), (40, 36)]:
            tr = oracle.pixel_trace(g, w.cams, P, 0, i, j)
            assert np.all(np.diff(tr["T"]) <= 0)
            assert tr["T"][0] == 1.0


def test_blend_order_is_mean_depth(oracle_lib):
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    g = oracle.Geometry.of(sc)
    Rm, tt, *_ = ref3d.cam_parts(w.cams[0])
    zt = ((sc.verts.astype(np.float64) @ Rm.T + tt)[:, 2])[sc.tets].mean(1)
    P = oracle.params_array(20.0, **EXACT)
    for (i, j) in [(32, 32), (26, 34)]:
        tr = oracle.pixel_trace(g, w.cams, P, 0, i, j)
        assert len(tr["tet"]) > 3
        assert np.all(np.diff(zt[tr["tet"]]) >= -1e-6)


def test_whole_image_matches_ray_route(oracle_lib):
    """Tiny image, float64: 2D barycentric route vs the independent 3D route."""
    w = synth.tiny(s=20.0, bg=(0.1, 0.2, 0.3))
    sc = w.scenes[0]
    g = oracle.Geometry.of(sc)
    for kw in ({}, EXACT):
        P = oracle.params_array(20.0, **kw)
        keep, *_ = oracle.prefilter(g, P)
        img = oracle.render_images(g, w.cams, P)[0]
        d = dict(oracle.DEFAULT, **kw)
        # thresholds travel as float32 parameters
        th = [float(np.float32(d[k])) for k in ("alpha_min", "alpha_clamp", "t_min")]
        ref, ties = ref3d.render_ray_route(sc.verts, sc.tets, sc.sdf, sc.colors, w.cams[0], 20.0,
                                           *th, keep)
        mask = np.ones(img.shape[1:], bool)
        for (i, j) in ties:
            mask[j, i] = False
        err = np.abs(img - ref)[:, mask].max()
        assert err < 1e-12, err
        assert mask.sum() > 4000


def test_large_s_sphere_silhouette(oracle_lib):
    verts, tets = synth.kuhn_grid(8)
    sdf = np.linalg.norm(verts, axis=1) - 0.5
    g = oracle.Geometry(verts, tets, sdf, np.full_like(verts, 0.5))
    cam = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, 64, 64)
    img = oracle.render_images(g, cam[None], oracle.params_array(2000.0))[0]
    jj, ii = np.meshgrid(np.arange(64) + 0.5, np.arange(64) + 0.5, indexing="ij")
    r = np.hypot(ii - 32, jj - 32)
    r_disk = cam[14] * math.tan(math.asin(0.5 / 2.5))   # 14.01 px
    assert 13.9 < r_disk < 14.1
    assert img[3][r < r_disk - 1.5].min() > 0.99
    assert img[3][r > r_disk + 1.0].max() < 0.01


# ---------------------------------------------------------------------------
# Binning (Sec. 3.3): brute force on the tiny grid
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tw,th", [(16, 16), (8, 8), (32, 8)])
def test_binning_brute_force(oracle_lib, tw, th):
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    g = oracle.Geometry.of(sc)
    P = oracle.params_array(20.0, tile_w=tw, tile_h=th)
    b = oracle.binning(g, w.cams, P, want_rect=True)
    W = H = 64
    ntx, nty = (W + tw - 1) // tw, (H + th - 1) // th
    rect = b["rect"][0]
    Rm, tt, fx, fy, cx, cy = ref3d.cam_parts(w.cams[0])
    Xc = sc.verts.astype(np.float64) @ Rm.T + tt
    zt32 = Xc[:, 2][sc.tets].mean(1)
    ents = []
    keep, *_ = oracle.prefilter(g, P)
    for k in np.nonzero(keep)[0]:
        i0, i1, j0, j1 = rect[k]
        if i0 < 0:
            continue
        # the rectangle is the set of pixel centres inside the projected bbox
        px = fx * Xc[sc.tets[k], 0] / Xc[sc.tets[k], 2] + cx
        py = fy * Xc[sc.tets[k], 1] / Xc[sc.tets[k], 2] + cy
        for i in range(W):
            inb = px.min() <= i + 0.5 <= px.max()
            if abs(i + 0.5 - px.min()) > 1e-4 and abs(i + 0.5 - px.max()) > 1e-4:
                assert inb == (i0 <= i <= i1)
        for ty in range(nty):
            for tx in range(ntx):
                if tx * tw <= i1 and i0 < (tx + 1) * tw and ty * th <= j1 and j0 < (ty + 1) * th:
                    ents.append((ty * ntx + tx, zt32[k], int(k)))
    ents.sort(key=lambda e: (e[0], e[1], e[2]))
    assert b["E"] == len(ents)
    assert np.array_equal(b["tile"], [e[0] for e in ents])
    # depth order from float64 depths agrees except on float32 ties
    same = np.array([e[2] for e in ents]) == b["tet"]
    assert same.mean() > 0.99
    # float32 keys are sorted within each tile, ties by tet id
    key = b["tile"].astype(np.int64) << 32 | b["zbits"].astype(np.int64)
    assert np.all(np.diff(key) >= 0)
    tie = np.diff(key) == 0
    assert np.all(np.diff(b["tet"])[tie] > 0)
    # ranges partition [0, E)
    r = b["ranges"]
    nonempty = r[:, 1] > r[:, 0]
    assert r[nonempty, 0].min() == 0 and r[nonempty, 1].max() == b["E"]
    assert (r[:, 1] - r[:, 0]).sum() == b["E"]
    # conservative: every tet that the per-pixel loop blends is in that pixel's tile list
    for (i, j) in [(32, 32), (25, 40), (38, 22)]:
        tr = oracle.pixel_trace(g, w.cams, oracle.params_array(20.0, tile_w=tw, tile_h=th, **EXACT), 0, i, j)
        t_id = (j // th) * ntx + (i // tw)
        lst = b["tet"][r[t_id, 0]:r[t_id, 1]]
        assert set(tr["tet"]).issubset(set(lst))
        # and the blend order is the tile order restricted to the pixel
        pos = [int(np.nonzero(lst == k)[0][0]) for k in tr["tet"]]
        assert pos == sorted(pos)


# ---------------------------------------------------------------------------
# Gradients: forward-mode duals and central finite differences (FP64)
# ---------------------------------------------------------------------------
def _visible_vertices(g, w, P, rng, n):
    out = oracle.render(g, w.cams, P)
    pix = oracle.all_pixels(w.cams)
    hot = pix[out[:, 3] > 0.05]
    vs = set()
    for (v, i, j) in hot[rng.choice(hot.shape[0], 40, replace=False)]:
        tr = oracle.pixel_trace(g, w.cams, P, int(v), int(i), int(j))
        for k in tr["tet"][:3]:
            vs.update(g.tets[k].tolist())
    vs = sorted(vs)
    return rng.choice(vs, min(n, len(vs)), replace=False)


@pytest.mark.parametrize("mode", ["exact", "default"])
def test_reverse_mode_matches_dual_numbers(oracle_lib, mode):
    w = synth.tiny(s=20.0, bg=(0.3, 0.1, 0.2))
    g = oracle.Geometry.of(w.scenes[0])
    P = oracle.params_array(20.0, **(EXACT if mode == "exact" else {}))
    pix = oracle.all_pixels(w.cams)
    rng = np.random.default_rng(21)
    wout = rng.normal(size=(pix.shape[0], 8))
    dv, ds, dc = oracle.backward(g, w.cams, P, pix, wout)
    for trial in range(3):
        tv = rng.normal(size=(g.V, 3))
        ts = rng.normal(size=g.V)
        tc = rng.normal(size=(g.V, 3))
        _, tout = oracle.render_dual(g, w.cams, P, pix, tv, ts, tc)
        lhs = float((wout * tout).sum())
        rhs = float((dv * tv).sum() + (ds * ts).sum() + (dc * tc).sum())
        assert lhs == pytest.approx(rhs, rel=1e-10)
        # each input group separately
        for args, grad, tan in (((tv, None, None), dv, tv), ((None, ts, None), ds, ts), ((None, None, tc), dc, tc)):
            _, t1 = oracle.render_dual(g, w.cams, P, pix, *args)
            assert float((wout * t1).sum()) == pytest.approx(float((grad * tan).sum()), rel=1e-10)


def test_gradient_central_differences(oracle_lib):
    w = synth.tiny(s=20.0, bg=(0.3, 0.1, 0.2))
    sc = w.scenes[0]
    g = oracle.Geometry.of(sc)
    P = oracle.params_array(20.0, **EXACT)
    pix = oracle.all_pixels(w.cams)
    rng = np.random.default_rng(31)
    wout = rng.normal(size=(pix.shape[0], 8))
    dv, ds, dc = oracle.backward(g, w.cams, P, pix, wout)
    verts = _visible_vertices(g, w, P, rng, 12)

    def loss(gg):
        return float((oracle.render(gg, w.cams, P, pix) * wout).sum())

    checked = 0
    for vi in verts:
        for what in ("sdf", "x", "y", "z", "r"):
            gp = oracle.Geometry(g.verts.copy(), g.tets, g.sdf.copy(), g.colors.copy())
            gm = oracle.Geometry(g.verts.copy(), g.tets, g.sdf.copy(), g.colors.copy())
            if what == "sdf":
                h = 1e-6
                gp.sdf[vi] += h; gm.sdf[vi] -= h
                ana = ds[vi]
            elif what == "r":
                h = 1e-3
                gp.colors[vi, 0] += h; gm.colors[vi, 0] -= h
                ana = dc[vi, 0]
            else:
                c = "xyz".index(what)
                h = 1e-6
                gp.verts[vi, c] += h; gm.verts[vi, c] -= h
                ana = dv[vi, c]
            fd = (loss(gp) - loss(gm)) / (2 * h)
            assert fd == pytest.approx(ana, rel=2e-4, abs=2e-4 * (abs(ana) + 1e-2)), (vi, what, fd, ana)
            checked += 1
    assert checked >= 50


def test_float32_oracle_close_to_float64(oracle_lib):
    w = synth.tiny(s=100.0)
    g = oracle.Geometry.of(w.scenes[0])
    P = oracle.params_array(100.0, **EXACT)
    a = oracle.render_images(g, w.cams, P, prec=32)[0]
    b = oracle.render_images(g, w.cams, P, prec=64)[0]
    assert np.abs(a - b).max() < 1e-4


# ---------------------------------------------------------------------------
# error budget of a float32 backward (the element-wise gradient bound of the
# GPU tests is built from it)
# ---------------------------------------------------------------------------
def _gamma(n):
    u = 2.0 ** -24
    return n * u / (1.0 - n * u)


def test_alpha_running_error_bound(oracle_lib):
    """The running error bound of Eq. 1 covers the float32 evaluation's actual
    error on random float32 inputs, and is not vacuous."""
    rng = np.random.default_rng(51)
    worst, rel = 0.0, []
    for s in (20.0, 320.0, 2000.0):
        fp = rng.uniform(-0.05, 0.05, 4000).astype(np.float32)
        fn = (fp - rng.uniform(0.0, 0.03, 4000)).astype(np.float32)
        for a_, b_ in zip(fp, fn):
            v, e = oracle.alpha_error_bound(a_, b_, s)
            err = abs(oracle.alpha_f32(a_, b_, s) - v)
            assert err <= e, (a_, b_, s, err, e)
            if v > 1e-3:
                rel.append(e / v)
    assert np.median(rel) < 1e-4


@pytest.mark.parametrize("s", [20.0, 100.0])
def test_forward_running_error_bound(oracle_lib, s):
    """Every channel of every pixel of the float32 oracle lies within the
    running error bound of the float64 value (exact mode: the walks blend the
    same tets except where float32 T reaches exactly 0)."""
    w = synth.tiny(s=s, bg=(0.3, 0.1, 0.2))
    g = oracle.Geometry.of(w.scenes[0])
    P = oracle.params_array(s, **EXACT)
    pix = oracle.all_pixels(w.cams)
    v, e = oracle.render_error_bound(g, w.cams, P, pix)
    assert np.array_equal(v, oracle.render(g, w.cams, P, pix, prec=64))
    r32, nb32, _ = oracle.render(g, w.cams, P, pix, prec=32, want_state=True)
    _, nb64, _ = oracle.render(g, w.cams, P, pix, prec=64, want_state=True)
    same = nb32 == nb64
    assert same.mean() > 0.9
    assert np.all(np.abs(r32 - v)[same] <= e[same])
    covered = v[:, 3] > 0.1
    assert np.median(e[covered & same, 0]) < 1e-3   # a few hundred units of u on O(1) colours


@pytest.mark.parametrize("s", [20.0, 100.0])
@pytest.mark.parametrize("mode", ["exact", "default"])
def test_backward_budget(oracle_lib, mode, s):
    """The float32 oracle's own error obeys its budget element by element; A
    bounds the float64 gradient (triangle inequality); an element no term
    reaches is exactly zero.  The colour part of A and N is recomputed from
    per-pixel traces (a colour term is 0.25 T alpha dL/dRGB per vertex of the
    blended tet), and its E is at least the float32 oracle's actual error in
    those terms, fl(fl(T a) g) against T a g."""
    w = synth.tiny(s=s, bg=(0.3, 0.1, 0.2))
    g = oracle.Geometry.of(w.scenes[0])
    P = oracle.params_array(s, **(EXACT if mode == "exact" else {}))
    allpix = oracle.all_pixels(w.cams)
    rng = np.random.default_rng(41)
    pix = allpix[rng.choice(allpix.shape[0], 300, replace=False)]
    dout = rng.normal(size=(pix.shape[0], 8)).astype(np.float32).astype(np.float64)
    r32 = oracle.backward(g, w.cams, P, pix, dout, prec=32)
    r64 = oracle.backward(g, w.cams, P, pix, dout, prec=64)
    b = oracle.backward_budget(g, w.cams, P, pix, dout)
    for k in range(3):
        A, E, N = b["A"][k], b["E"][k], b["N"][k]
        err = np.abs(r32[k] - r64[k])
        assert np.all(err <= E + _gamma(N + 32) * A), k
        assert np.all(np.abs(r64[k]) <= A * (1 + 1e-12)), k
        none = N == 0
        assert np.all(A[none] == 0) and np.all(E[none] == 0)
        assert np.all(r32[k][none] == 0) and np.all(r64[k][none] == 0)
    # colour part from traces
    Ac = np.zeros((g.V, 3))
    Ec = np.zeros((g.V, 3))
    Nc = np.zeros(g.V)
    for (v, i, j), d in zip(pix, dout):
        t64 = oracle.pixel_trace(g, w.cams, P, int(v), int(i), int(j), prec=64)
        t32 = oracle.pixel_trace(g, w.cams, P, int(v), int(i), int(j), prec=32)
        # the precisions may blend different lists (in exact mode float32 alpha
        # can round to 1 and end the walk): a term of one list only counts in full
        w64 = {int(t): T * a for t, T, a in zip(t64["tet"], t64["T"], t64["alpha"])}
        w32 = {int(t): np.float32(np.float32(T) * np.float32(a)) for t, T, a in zip(t32["tet"], t32["T"], t32["alpha"])}
        for tet in set(w64) | set(w32):
            g32 = (w32[tet] * d[:3].astype(np.float32)).astype(np.float64) if tet in w32 else np.zeros(3)
            g64 = w64[tet] * d[:3] if tet in w64 else np.zeros(3)
            for vi in g.tets[tet]:
                Ac[vi] += 0.25 * np.maximum(np.abs(g32), np.abs(g64))
                Ec[vi] += 0.25 * np.abs(g32 - g64)
                Nc[vi] += 1
    np.testing.assert_allclose(b["A"][2], Ac, rtol=1e-12, atol=0)
    assert np.all(b["E"][2] >= Ec)
    assert np.array_equal(b["N"][2][:, 0], Nc)
    assert Nc.max() > 1 and np.count_nonzero(Ec) > 0


def test_pixel_decisions_follow_the_walk(oracle_lib):
    """The decision log of a pixel lists every candidate's skip test, then per
    blended tet its clamp and stop tests (the stopping tet's stop test last);
    its float64 values are the walk's own and the float32 walk's values lie
    within their running bounds."""
    w = synth.tiny(s=100.0)
    g = oracle.Geometry.of(w.scenes[0])
    P = oracle.params_array(100.0)
    out = oracle.render(g, w.cams, P)
    pix = oracle.all_pixels(w.cams)
    hot = pix[out[:, 3] > 0.05]
    rng = np.random.default_rng(61)
    stopped = 0
    for (v, i, j) in hot[rng.choice(hot.shape[0], 150, replace=False)]:
        d = oracle.pixel_decisions(g, w.cams, P, v, i, j)
        t64 = oracle.pixel_trace(g, w.cams, P, v, i, j, prec=64)
        t32 = oracle.pixel_trace(g, w.cams, P, v, i, j, prec=32)
        nb = len(t64["tet"])
        k = d["kind"]
        n0 = int(np.sum(k == 0))
        assert np.all(k[:n0] == 0) and np.all(k[n0:][0::2] == 1) and np.all(k[n0:][1::2] == 2)
        assert n0 >= nb and np.sum(k == 2) in (nb, nb + 1)
        stopped += int(np.sum(k == 2) == nb + 1)
        a_cl = d["value"][n0:][0::2][:nb]
        assert np.array_equal(a_cl, t64["alpha_raw"])
        # T (1 - alpha) of a blended tet is the next tet's T
        tn = d["value"][n0:][1::2][:nb - 1]
        assert np.allclose(tn, t64["T"][1:], rtol=1e-15, atol=0)
        if np.array_equal(t32["tet"], t64["tet"]):
            assert np.all(np.abs(t32["alpha_raw"] - a_cl) <= d["bound"][n0:][0::2][:nb])
    assert stopped > 0
