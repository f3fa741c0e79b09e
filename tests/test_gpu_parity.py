"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: tile ids, per-tile ranges and
sort order bit-exact; images within 1e-5 max-abs and gradients within 1e-4
relative (|g-r| / (|r| + 1e-3 max|r|)) of the float32 oracle.  The error
against the float64 oracle is printed per output.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import (IMG_TOL, check_gradients, oracle_gradients, compare_images, gpu_forward, gpu_tiling,
                               oracle_params)

pytestmark = pytest.mark.gpu

TILES = [(8, 8), (16, 8), (8, 16), (16, 16), (32, 8)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _params(mode, tile=(16, 16), **kw):
    from paper_2406_01579_amd import Params
    base = Params.exact if mode == "exact" else Params
    return base(tile_w=tile[0], tile_h=tile[1], **kw)


# ---------------------------------------------------------------------------
# tiny grid: full images, full tiling, full gradients
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("s", [20.0, 100.0])
@pytest.mark.parametrize("mode", ["exact", "default"])
def test_tiny_images(mode, s):
    w = synth.tiny(s=s, bg=(0.1, 0.2, 0.3))
    sc = w.scenes[0]
    P = _params(mode)
    _, _, imgs = gpu_forward(sc, w.cams, P)
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, s)
    err32, n_ex, n = compare_images(imgs, g, w.cams, op, s)
    err64 = np.abs(imgs[0] - oracle.render_images(g, w.cams, op, prec=64)[0]).reshape(8, -1).max(1)
    print(f"tiny {mode} s={s}: max-abs vs f32 {err32:.3e} (excluded {n_ex}/{n}); vs f64 per channel {err64}")
    assert err32 <= IMG_TOL
    assert n_ex <= max(1, int(1e-4 * n))


@pytest.mark.parametrize("tile", TILES)
def test_tiny_tiling_bit_exact(tile):
    s = 20.0
    w = synth.tiny(s=s)
    sc = w.scenes[0]
    P = _params("default", tile)
    r, plan, _ = gpu_forward(sc, w.cams, P)
    d, tets = gpu_tiling(r, plan)
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, s)
    keep, *_ = oracle.prefilter(g, op)
    assert np.array_equal(np.sort(d["kept_tet"]), np.nonzero(keep)[0])
    assert np.all(np.diff(d["kept_tet"]) > 0)  # compaction keeps ascending tet order
    ref = oracle.binning(g, w.cams, op)
    assert d["entries"] == ref["E"]
    assert np.array_equal(d["tile_keys"], ref["tile"].astype(np.uint32))
    assert np.array_equal(tets, ref["tet"])
    assert np.array_equal(d["ranges"].astype(np.int64), ref["ranges"].astype(np.int64))


@pytest.mark.parametrize("tile", TILES)
def test_tile_shape_does_not_change_image(tile):
    """Per-pixel blend order and arithmetic do not depend on the tiling."""
    w = synth.tiny(s=100.0, bg=(0.3, 0.3, 0.3))
    _, _, a = gpu_forward(w.scenes[0], w.cams, _params("default", (16, 16)))
    _, _, b = gpu_forward(w.scenes[0], w.cams, _params("default", tile))
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("recompute", [False, True])
@pytest.mark.parametrize("s", [20.0, 100.0])
@pytest.mark.parametrize("mode", ["exact", "default"])
@pytest.mark.parametrize("tile", TILES)
def test_tiny_gradients(tile, mode, s, recompute):
    """Every tile shape the autotuner may pick (8x8 with four waves per tile)."""
    import torch
    w = synth.tiny(s=s, bg=(0.3, 0.1, 0.2))
    sc = w.scenes[0]
    P = _params(mode, tile, recompute_state=recompute)
    r, plan, _ = gpu_forward(sc, w.cams, P)
    rng = np.random.default_rng(5)
    dout = rng.normal(size=(8, 64, 64)).astype(np.float32)
    (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
    torch.cuda.synchronize()
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, s)
    pix = oracle.all_pixels(w.cams)
    dflat = dout.reshape(8, -1).T.copy()
    refs = oracle_gradients(g, w.cams, op, pix, dflat)
    check_gradients((dv, ds, dc), refs, f"tiny {tile} {mode} s={s} recompute={recompute}")


def _tuner_candidates():
    from paper_2406_01579_amd import tune
    return tune.candidates(), [tune.label(c) for c in tune.candidates()]


@pytest.mark.parametrize("cand", _tuner_candidates()[0], ids=_tuner_candidates()[1])
def test_every_tuner_candidate_against_the_oracle(cand):
    """Every launch shape the autotuner may pick (tile, waves per 8x8 tile,
    forward and backward LDS chunk lengths): images of the tiny grid against
    the oracle, and the gradients of a dense upstream gradient on it and on a
    ragged image, with stored and with recomputed per-pixel state."""
    import torch
    tw, th, wv, cf, cb = cand
    s = 100.0
    w = synth.tiny(s=s, bg=(0.3, 0.1, 0.2))
    sc = w.scenes[0]
    g = oracle.Geometry.of(sc)
    Wd, Hd = 130, 9
    rag = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, Wd, Hd, bg=(0.2, 0.5, 0.1))[None]
    rag[0, 17] = Hd / 2.0
    for cams, seed, rc in ((w.cams, 5, False), (rag, 21, True)):
        P = _params("default", (tw, th), waves=wv, chunk_fwd=cf, chunk_bwd=cb, recompute_state=rc)
        op = oracle_params(P, s)
        r, plan, imgs = gpu_forward(sc, cams, P)
        err32, n_ex, n = compare_images(imgs, g, cams, op, s)
        assert err32 <= IMG_TOL and n_ex <= max(1, int(1e-4 * n)), (cand, err32, n_ex)
        H, W = int(cams[0][1]), int(cams[0][0])
        dout = np.random.default_rng(seed).normal(size=(8, H, W)).astype(np.float32)
        (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
        torch.cuda.synchronize()
        pix = oracle.all_pixels(cams)
        dflat = np.stack([dout[:, j, i] for (_, i, j) in pix], 0).astype(np.float32)
        refs = oracle_gradients(g, cams, op, pix, dflat)
        check_gradients((dv, ds, dc), refs, f"candidate {cand} {W}x{H} recompute={rc}")


def test_recompute_state_matches_stored_state():
    import torch
    w = synth.tiny(s=100.0)
    sc = w.scenes[0]
    dout = torch.from_numpy(np.random.default_rng(6).normal(size=(8, 64, 64)).astype(np.float32)).cuda()
    res = []
    for rc in (False, True):
        r, plan, _ = gpu_forward(sc, w.cams, _params("default", recompute_state=rc))
        res.append([t.cpu().numpy() for t in r.backward(plan, [dout])[0]])
    for a, b in zip(*res):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(b).max())


# ---------------------------------------------------------------------------
# batches of views and scenes
# ---------------------------------------------------------------------------
def test_views_in_one_launch_equal_views_alone():
    w = synth.training(s=320.0, R=16, size=96, views=3)
    sc = w.scenes[0]
    P = _params("default")
    _, _, together = gpu_forward(sc, w.cams, P)
    for v in range(3):
        _, _, alone = gpu_forward(sc, w.cams[v:v + 1], P)
        assert np.array_equal(together[v], alone[0]), v


def test_scenes_of_uneven_size_in_one_launch():
    import torch
    from paper_2406_01579_amd import Renderer, SceneT
    rng = np.random.default_rng(9)
    scenes = [synth.scene_blob(R, rng, 320.0) for R in (12, 20, 8)]
    cams = synth.random_orbit_cameras(rng, 5, [64, 48, 80, 64, 40])
    vs = np.array([0, 1, 2, 1, 0], np.int32)
    P = _params("default")
    r = Renderer(P)
    sts = [SceneT.from_numpy(s) for s in scenes]
    plan = r.forward(sts, cams, vs)
    torch.cuda.synchronize()
    for v in range(5):
        p1 = Renderer(P).forward([sts[vs[v]]], cams[v:v + 1])
        torch.cuda.synchronize()
        assert np.array_equal(plan.outs[v].cpu().numpy(), p1.outs[0].cpu().numpy()), v
        g = oracle.Geometry.of(scenes[vs[v]])
        err, n_ex, n = compare_images([plan.outs[v].cpu().numpy()], g, cams[v:v + 1],
                                      oracle_params(P, 320.0), 320.0)
        assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n))
    # gradients of a multi-scene batch: each scene against the oracle
    douts = [torch.randn(o.shape, device="cuda") for o in plan.outs]
    grads = r.backward(plan, douts)
    torch.cuda.synchronize()
    for si, sc in enumerate(scenes):
        sel = [v for v in range(5) if vs[v] == si]
        pix = oracle.all_pixels(cams[sel])
        dflat = np.concatenate([douts[v].cpu().numpy().reshape(8, -1).T for v in sel], 0)
        gg = oracle.Geometry.of(sc)
        refs = oracle_gradients(gg, cams[sel], oracle_params(P, 320.0), pix, dflat)
        check_gradients(grads[si], refs, f"multi-scene scene {si}")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("size", [(1, 1), (50, 37), (8, 8), (130, 9)])
def test_ragged_image_sizes(size):
    s = 100.0
    w = synth.tiny(s=s, bg=(0.2, 0.5, 0.1))
    Wd, Hd = size
    cam = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, Wd, Hd, bg=(0.2, 0.5, 0.1))[None]
    cam[0, 17] = Hd / 2.0
    for tile in [(16, 16), (32, 8), (8, 8)]:
        P = _params("default", tile)
        _, _, imgs = gpu_forward(w.scenes[0], cam, P)
        err, n_ex, n = compare_images(imgs, oracle.Geometry.of(w.scenes[0]), cam, oracle_params(P, s), s)
        assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n)), (size, tile)


def test_vertex_gradients_without_shared_vertices():
    """A soup of small tets that share no vertex, seen from one view: every
    block of the vertex backward meets about a thousand distinct vertices,
    more than its LDS table holds, so most of them take the direct global
    atomics; the gradients must still match the oracle.  (On this soup the
    float32 and float64 oracles take some alpha_min / t_min decisions
    differently, so the normwise bar against the float32 oracle is the one
    that bites.)"""
    import torch
    rng = np.random.default_rng(44)
    K = 1024
    centres = rng.uniform(-0.45, 0.45, size=(K, 1, 3))
    verts = (centres + rng.normal(scale=0.04, size=(K, 4, 3))).reshape(-1, 3).astype(np.float32)
    tets = np.arange(4 * K, dtype=np.int32).reshape(K, 4)
    sdf = rng.uniform(-0.05, 0.05, size=4 * K).astype(np.float32)
    colors = rng.uniform(0.0, 1.0, size=(4 * K, 3)).astype(np.float32)
    s = 40.0
    sc = synth.Scene(verts, tets, sdf, colors, s, "soup")
    cam = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, 64, 64, (0.1, 0.2, 0.3))[None]
    for P in (_params("default", (8, 8), waves=4), _params("default")):
        r, plan, _ = gpu_forward(sc, cam, P)
        dout = rng.normal(size=(8, 64, 64)).astype(np.float32)
        (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
        torch.cuda.synchronize()
        g = oracle.Geometry.of(sc)
        op = oracle_params(P, s)
        pix = oracle.all_pixels(cam)
        dflat = dout.reshape(8, -1).T.copy()
        refs = oracle_gradients(g, cam, op, pix, dflat)
        check_gradients((dv, ds, dc), refs, f"tet soup tile {P.tile_w}x{P.tile_h}")


@pytest.mark.parametrize("recompute", [False, True])
@pytest.mark.parametrize("size", [(50, 37), (130, 9)])
@pytest.mark.parametrize("tile", TILES)
def test_ragged_image_gradients(tile, size, recompute):
    """Partial tiles at the right and bottom edges (including the tiles
    nothing reaches) through the backward of every tile shape, against the
    oracle."""
    import torch
    s = 100.0
    w = synth.tiny(s=s, bg=(0.2, 0.5, 0.1))
    Wd, Hd = size
    cam = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, Wd, Hd, bg=(0.2, 0.5, 0.1))[None]
    cam[0, 17] = Hd / 2.0
    P = _params("default", tile, recompute_state=recompute)
    r, plan, _ = gpu_forward(w.scenes[0], cam, P)
    dout = np.random.default_rng(21).normal(size=(8, Hd, Wd)).astype(np.float32)
    (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
    torch.cuda.synchronize()
    g = oracle.Geometry.of(w.scenes[0])
    op = oracle_params(P, s)
    pix = oracle.all_pixels(cam)
    dflat = np.stack([dout[:, j, i] for (_, i, j) in pix], 0).astype(np.float32)
    refs = oracle_gradients(g, cam, op, pix, dflat)
    check_gradients((dv, ds, dc), refs, f"ragged {tile} {size} recompute={recompute}")


def test_empty_scene_and_culled_views():
    import torch
    w = synth.tiny(s=20.0, bg=(0.25, 0.5, 0.75))
    sc = w.scenes[0]
    empty = synth.Scene(sc.verts, sc.tets, np.full_like(sc.sdf, 2.0), sc.colors, 20.0)
    # camera facing away from the grid: everything culled by the near plane / screen
    away = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, 64, 64, bg=(0.25, 0.5, 0.75))
    R = away[2:11].reshape(3, 3).astype(np.float64)
    C = -R.T @ away[11:14].astype(np.float64)      # camera centre
    R[2] *= -1
    R[0] *= -1
    away[2:11] = R.ravel()
    away[11:14] = -R @ C
    for scene, cams in ((empty, w.cams), (sc, away[None])):
        r, plan, imgs = gpu_forward(scene, cams, _params("default"))
        bg = np.array([0.25, 0.5, 0.75], np.float32)
        assert np.array_equal(imgs[0][0:3], np.broadcast_to(bg[:, None, None], (3, 64, 64)))
        assert np.all(imgs[0][3:] == 0)
        (dv, ds, dc), = r.backward(plan, [torch.ones(8, 64, 64, device="cuda")])
        assert float(dv.abs().max()) == 0 and float(ds.abs().max()) == 0 and float(dc.abs().max()) == 0
    # a scene with no tets at all
    none = synth.Scene(sc.verts, np.zeros((0, 4), np.int32), sc.sdf, sc.colors, 20.0)
    _, _, imgs = gpu_forward(none, w.cams, _params("default"))
    assert np.all(imgs[0][3:] == 0)


def test_out_of_range_indices_are_dropped_and_reported():
    import torch
    from paper_2406_01579_amd import Renderer, SceneT
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    bad = sc.tets.copy()
    bad[5, 2] = sc.V + 7
    bad[9, 0] = -3
    r = Renderer(_params("default"))
    with pytest.raises(ValueError, match="outside"):
        r.forward([SceneT.from_numpy(synth.Scene(sc.verts, bad, sc.sdf, sc.colors, 20.0))], w.cams)
    torch.cuda.synchronize()


def test_capacity_overflow_is_detected_and_replanned():
    import torch
    from paper_2406_01579_amd import Renderer, SceneT
    from paper_2406_01579_amd.frontend import CapacityError
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    P = _params("default")
    st = SceneT.from_numpy(sc)
    _, _, ref = gpu_forward(sc, w.cams, P)
    r = Renderer(P)
    sig = r._signature([st], w.cams, np.zeros(1, np.int32))
    r._caps[sig] = (2000, 10)       # far too few entries: the forward overflows, sync mode re-plans
    plan = r.forward([st], w.cams)
    assert plan.status.overflow == 0 and plan.entry_cap >= plan.status.entries
    assert np.array_equal(plan.outs[0].cpu().numpy(), ref[0])
    # lazy mode: the overflow surfaces before the backward, never silently
    r2 = Renderer(P, check="lazy")
    r2._caps[sig] = (2000, 10)
    plan2 = r2.forward([st], w.cams)
    with pytest.raises(CapacityError):
        r2.backward(plan2, [torch.zeros(8, 64, 64, device="cuda")])
    plan3 = r2.forward([st], w.cams)          # enlarged capacities now suffice
    r2.backward(plan3, [torch.zeros(8, 64, 64, device="cuda")])
    assert np.array_equal(plan3.outs[0].cpu().numpy(), ref[0])


def test_pair_overflow_keeps_the_forward_and_replans_the_backward():
    """Entries that fit while the (entry, pixel) pairs the forward blended do
    not (the multi-wave 8x8 backward keeps them in entry-capacity buffers):
    status bit 2 alone, the images stand, the backward is refused until the
    forward is re-planned, and the re-planned gradients equal those of a
    workspace sized from the start."""
    import torch
    from paper_2406_01579_amd import Renderer, SceneT
    from paper_2406_01579_amd.frontend import CapacityError
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    P = _params("exact", (8, 8), deterministic=True)   # every covered pixel blends: many pairs per entry
    st = SceneT.from_numpy(sc)
    r0, plan0, ref = gpu_forward(sc, w.cams, P)
    E = int(plan0.status.entries)
    dout = torch.from_numpy(np.random.default_rng(3).normal(size=(8, 64, 64)).astype(np.float32)).cuda()
    (g0,) = r0.backward(plan0, [dout])
    g0 = [t.cpu().numpy() for t in g0]
    r = Renderer(P, check="lazy")
    sig = r._signature([st], w.cams, np.zeros(1, np.int32))
    r._caps[sig] = (sc.K, E + 16)
    plan = r.forward([st], w.cams)
    torch.cuda.synchronize()
    s1 = r.read_status(plan)
    assert s1.overflow == 4 and s1.entries == E and s1.entries_needed > E + 16
    assert np.array_equal(plan.outs[0].cpu().numpy(), ref[0])
    with pytest.raises(CapacityError):
        r.backward(plan, [dout])
    plan2 = r.forward([st], w.cams)            # enlarged to the pairs it needs
    torch.cuda.synchronize()
    assert r.read_status(plan2).overflow == 0 and plan2.entry_cap >= s1.entries_needed
    (g2,) = r.backward(plan2, [dout])
    for a, b in zip(g2, g0):
        assert np.array_equal(a.cpu().numpy(), b)


def test_capacities_sized_from_a_forward_cover_its_pairs():
    """The status's entries_needed covers the blended pairs when they are more
    than the entries, so capacities sized from a first forward leave the
    backward room for its pairs: later lazy-checked steps never overflow."""
    import torch
    from paper_2406_01579_amd import Renderer, SceneT
    w = synth.tiny(s=20.0)
    sc = w.scenes[0]
    st = SceneT.from_numpy(sc)
    r = Renderer(_params("exact", (8, 8)), check="lazy")
    plan = r.forward([st], w.cams)        # first sight of the shape: sized synchronously
    s = plan.status
    assert s.overflow == 0 and s.entries_needed > s.entries   # more pairs than entries here
    dout = torch.zeros(8, 64, 64, device="cuda")
    r.backward(plan, [dout])
    for _ in range(3):
        plan = r.forward([st], w.cams)
        r.backward(plan, [dout])
    torch.cuda.synchronize()
    assert r.read_status(plan).overflow == 0


# ---------------------------------------------------------------------------
# training-shaped workload at full size (64^3 grid, 4 views 512^2, s = 320):
# tiling in full, sampled pixels, gradients of a sparse upstream gradient
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def training():
    w = synth.training(s=320.0)
    return w, oracle.Geometry.of(w.scenes[0])


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_training_tiling_bit_exact(training, tile):
    w, g = training
    P = _params("default", tile)
    r, plan, _ = gpu_forward(w.scenes[0], w.cams, P)
    d, tets = gpu_tiling(r, plan)
    op = oracle_params(P, 320.0)
    keep, amax, *_ = oracle.prefilter(g, op)
    gk = np.zeros(g.K, bool)
    gk[d["kept_tet"]] = True
    diff = np.nonzero(gk != keep)[0]
    # a kept-set difference may only come from exp/expm1 rounding at T_f
    tf = np.float32(1 / 255)
    assert np.all(np.abs(amax[diff] - tf) <= 4 * np.spacing(tf)), diff
    ref = oracle.binning(g, w.cams, op)
    if diff.size == 0:
        assert d["entries"] == ref["E"]
        assert np.array_equal(d["tile_keys"], ref["tile"].astype(np.uint32))
        assert np.array_equal(tets, ref["tet"])
        assert np.array_equal(d["ranges"].astype(np.int64), ref["ranges"].astype(np.int64))
    else:
        m_gpu = ~np.isin(tets, diff)
        m_ref = ~np.isin(ref["tet"], diff)
        assert np.array_equal(d["tile_keys"][m_gpu], ref["tile"][m_ref].astype(np.uint32))
        assert np.array_equal(tets[m_gpu], ref["tet"][m_ref])
    print(f"training tiling {tile}: E={d['entries']}, kept={d['kept']}, kept-set differences {diff.size}")


def _sample_pixels(w, n, seed):
    rng = np.random.default_rng(seed)
    nv = w.cams.shape[0]
    W, H = int(w.cams[0, 0]), int(w.cams[0, 1])
    pix = np.stack([rng.integers(0, nv, n), rng.integers(0, W, n), rng.integers(0, H, n)], 1)
    return np.ascontiguousarray(pix, dtype=np.int32)


@pytest.mark.parametrize("mode", ["exact", "default"])
def test_training_sampled_pixels(training, mode):
    w, g = training
    P = _params(mode)
    _, _, imgs = gpu_forward(w.scenes[0], w.cams, P)
    pix = _sample_pixels(w, 3000, 1)
    # bias the sample toward the object: half of it from covered pixels
    cov = np.argwhere(np.stack(imgs)[:, 3] > 0.01)
    pick = cov[np.random.default_rng(2).choice(len(cov), 1500, replace=False)]
    pix = np.concatenate([pix, pick[:, [0, 2, 1]].astype(np.int32)], 0)
    op = oracle_params(P, 320.0)
    err, n_ex, n = compare_images(imgs, g, w.cams, op, 320.0, pix=pix)
    got = np.stack([imgs[v][:, j, i] for (v, i, j) in pix], 0)
    e64 = np.abs(got - oracle.render(g, w.cams, op, pix, prec=64)).max(0)
    print(f"training {mode}: sampled max-abs vs f32 {err:.3e} (excluded {n_ex}/{n}); vs f64 per channel {e64}")
    assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n))


def test_training_gradients_of_sparse_upstream(training):
    """dL/dout nonzero on a pixel sample only: the oracle computes that
    backward exactly at full size."""
    import torch
    w, g = training
    P = _params("default")
    r, plan, imgs = gpu_forward(w.scenes[0], w.cams, P)
    cov = np.argwhere(np.stack(imgs)[:, 3] > 0.01)
    pick = cov[np.random.default_rng(3).choice(len(cov), 2000, replace=False)]
    pix = np.ascontiguousarray(pick[:, [0, 2, 1]], dtype=np.int32)
    rng = np.random.default_rng(4)
    vals = rng.normal(size=(pix.shape[0], 8)).astype(np.float32)
    douts = [np.zeros((8, 512, 512), np.float32) for _ in range(4)]
    for (v, i, j), x in zip(pix, vals):
        douts[v][:, j, i] += x
    # merge duplicates the same way for the oracle
    key = pix[:, 0] * 512 * 512 + pix[:, 2] * 512 + pix[:, 1]
    uk, first = np.unique(key, return_index=True)
    upix = pix[first]
    dflat = np.stack([douts[v][:, j, i] for (v, i, j) in upix], 0).astype(np.float64)
    grads, = r.backward(plan, [torch.from_numpy(d).cuda() for d in douts])
    torch.cuda.synchronize()
    op = oracle_params(P, 320.0)
    refs = oracle_gradients(g, w.cams, op, upix, dflat)
    check_gradients(grads, refs, "training sparse-upstream")


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_waves_per_tile_do_not_change_results(waves):
    """Several waves sharing an 8x8 tile evaluate the same per-pair arithmetic."""
    import torch
    w = synth.tiny(s=100.0, bg=(0.3, 0.3, 0.3))
    sc = w.scenes[0]
    dout = torch.from_numpy(np.random.default_rng(8).normal(size=(8, 64, 64)).astype(np.float32)).cuda()
    res = []
    for wv in (1, waves):
        for rc in (False, True):
            r, plan, imgs = gpu_forward(sc, w.cams, _params("default", (8, 8), waves=wv, recompute_state=rc))
            grads = [t.cpu().numpy() for t in r.backward(plan, [dout])[0]]
            res.append((imgs[0], grads))
    ref_img, ref_g = res[0]
    for img, grads in res[1:]:
        assert np.array_equal(img, ref_img)
        for a, b in zip(grads, ref_g):
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(b).max())


# ---------------------------------------------------------------------------
# the training-shaped workload in the launch configuration the benchmark
# times (8x8 tiles, four waves per tile): every pixel of all four views, and
# the gradient of a dense upstream gradient on every pixel
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["exact", "default"])
def test_training_full_images_timed_shape(training, mode):
    w, g = training
    P = _params(mode, (8, 8), waves=4)
    _, _, imgs = gpu_forward(w.scenes[0], w.cams, P)
    op = oracle_params(P, 320.0)
    err, n_ex, n = compare_images(imgs, g, w.cams, op, 320.0)
    pix = _sample_pixels(w, 20000, 12)
    got = np.stack([imgs[v][:, j, i] for (v, i, j) in pix], 0)
    e64 = np.abs(got - oracle.render(g, w.cams, op, pix, prec=64)).max(0)
    print(f"training 8x8/4 waves {mode}: all {n} pixels max-abs vs f32 {err:.3e} (excluded {n_ex}); "
          f"vs f64 per channel (20000 sampled) {e64}")
    assert n == 4 * 512 * 512
    assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n))


def test_training_gradients_dense_upstream_timed_shape(training):
    import torch
    w, g = training
    P = _params("default", (8, 8), waves=4)
    r, plan, _ = gpu_forward(w.scenes[0], w.cams, P)
    douts = np.random.default_rng(13).normal(size=(4, 8, 512, 512)).astype(np.float32)
    grads, = r.backward(plan, [torch.from_numpy(d).cuda() for d in douts])
    torch.cuda.synchronize()
    pix = oracle.all_pixels(w.cams)
    dflat = douts.transpose(0, 2, 3, 1).reshape(-1, 8).astype(np.float64)
    # all_pixels lists each view row by row (j outer, i inner): the same order
    assert np.array_equal(pix[:3, 1], [0, 1, 2]) and pix[512, 2] == 1
    refs = oracle_gradients(g, w.cams, oracle_params(P, 320.0), pix, dflat)
    check_gradients(grads, refs, "training 8x8/4 waves dense upstream")


# ---------------------------------------------------------------------------
# memory and reproducibility modes of the backward
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["record_grads", "deterministic", "record_grads+recompute"])
@pytest.mark.parametrize("tile", TILES)
def test_tiny_gradients_backward_modes(tile, mode):
    """Per-record gradient accumulators, the deterministic reductions and the
    recomputed per-pixel state against the oracle, for every tile shape."""
    import torch
    s = 100.0
    w = synth.tiny(s=s, bg=(0.3, 0.1, 0.2))
    sc = w.scenes[0]
    P = _params("default", tile, record_grads="record_grads" in mode, deterministic=mode == "deterministic",
                recompute_state="recompute" in mode)
    r, plan, _ = gpu_forward(sc, w.cams, P)
    dout = np.random.default_rng(5).normal(size=(8, 64, 64)).astype(np.float32)
    (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
    torch.cuda.synchronize()
    g = oracle.Geometry.of(sc)
    pix = oracle.all_pixels(w.cams)
    refs = oracle_gradients(g, w.cams, oracle_params(P, s), pix, dout.reshape(8, -1).T.copy())
    check_gradients((dv, ds, dc), refs, f"tiny {tile} {mode}")


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_training_deterministic_gradients_are_bitwise_repeatable(training, tile):
    """RENDER_DETERMINISTIC: three backward passes of one forward and a
    second forward + backward give bitwise-identical gradients, equal to the
    default mode's to rounding."""
    import torch
    w, g = training
    douts = [torch.from_numpy(d).cuda()
             for d in np.random.default_rng(17).normal(size=(4, 8, 512, 512)).astype(np.float32)]
    P = _params("default", tile, deterministic=True)
    r, plan, _ = gpu_forward(w.scenes[0], w.cams, P)
    runs = []
    for _ in range(3):
        runs.append([t.cpu().numpy() for t in r.backward(plan, douts)[0]])
    r2, plan2, _ = gpu_forward(w.scenes[0], w.cams, P)
    runs.append([t.cpu().numpy() for t in r2.backward(plan2, douts)[0]])
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert np.array_equal(a, b)
    rd, pd, _ = gpu_forward(w.scenes[0], w.cams, _params("default", tile))
    ref = [t.cpu().numpy() for t in rd.backward(pd, douts)[0]]
    for name, a, b in zip(("dverts", "dsdf", "dcolors"), runs[0], ref):
        n = float(np.abs(a - b).max() / np.abs(b).max())
        print(f"deterministic {tile} {name}: normwise vs default mode {n:.2e}")
        assert n <= 1e-5


@pytest.mark.parametrize("waves,chunks", [(2, (32, 16)), (4, (64, 32)), (8, (64, 32))])
def test_multiwave_gradients_repeat_bitwise(waves, chunks):
    """The multi-wave 8x8 backward with 2, 4 and 8 waves per tile, run eight
    times on one input (deterministic mode: every sum in a fixed order): the
    gradients are bit for bit equal, so no repeat sees another wave's LDS
    or global hand-over early (the chunk arrays, candidate masks, pair
    places and blend masks pass between waves only across barriers or
    kernel boundaries)."""
    import torch
    w = synth.training(s=320.0, R=16, size=96, views=2)
    sc = w.scenes[0]
    P = _params("default", (8, 8), waves=waves, chunk_fwd=chunks[0], chunk_bwd=chunks[1], deterministic=True)
    gen = np.random.default_rng(13)
    douts = [torch.from_numpy(gen.normal(size=(8, 96, 96)).astype(np.float32)).cuda() for _ in range(2)]
    r, plan, img0 = gpu_forward(sc, w.cams, P)
    ref = [t.cpu().numpy() for t in r.backward(plan, douts)[0]]
    assert max(np.abs(t).max() for t in ref) > 0
    for _ in range(7):
        r, plan, img = gpu_forward(sc, w.cams, P)
        assert all(np.array_equal(a, b) for a, b in zip(img, img0))
        got = [t.cpu().numpy() for t in r.backward(plan, douts)[0]]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_training_record_grads_and_recomputed_state_shrink_the_workspace(training):
    """RENDER_RECORD_GRADS + RENDER_RECOMPUTE_STATE at the training shape:
    a smaller workspace, the same image, gradients of a sparse upstream
    gradient against the oracle and equal to the default mode's to rounding."""
    import torch
    w, g = training
    Pd = _params("default", (8, 8))
    Pm = _params("default", (8, 8), record_grads=True, recompute_state=True)
    rd, pd, imd = gpu_forward(w.scenes[0], w.cams, Pd)
    rm, pm, imm = gpu_forward(w.scenes[0], w.cams, Pm)
    for a, b in zip(imd, imm):
        assert np.array_equal(a, b)
    caps = rm.capacity(pm.scenes, w.cams)   # the capacities sized by the first forward
    nd = rd.workspace_bytes(pd.scene_c, pd.view_c, pd.params_c, *caps)
    nm = rm.workspace_bytes(pm.scene_c, pm.view_c, pm.params_c, *caps)
    print(f"workspace at the same capacities {caps}: default {nd / 2**20:.1f} MiB, record grads + recomputed "
          f"state {nm / 2**20:.1f} MiB")
    assert nm < 0.75 * nd
    cov = np.argwhere(np.stack(imd)[:, 3] > 0.01)
    pick = cov[np.random.default_rng(3).choice(len(cov), 2000, replace=False)]
    pix = np.ascontiguousarray(pick[:, [0, 2, 1]], dtype=np.int32)
    key = pix[:, 0] * 512 * 512 + pix[:, 2] * 512 + pix[:, 1]
    _, first = np.unique(key, return_index=True)
    upix = pix[first]
    vals = np.random.default_rng(4).normal(size=(upix.shape[0], 8)).astype(np.float32)
    douts = [np.zeros((8, 512, 512), np.float32) for _ in range(4)]
    for (v, i, j), x in zip(upix, vals):
        douts[v][:, j, i] = x
    dt = [torch.from_numpy(d).cuda() for d in douts]
    gm = rm.backward(pm, dt)[0]
    gd = rd.backward(pd, dt)[0]
    torch.cuda.synchronize()
    for name, a, b in zip(("dverts", "dsdf", "dcolors"), gm, gd):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert float(np.abs(a - b).max() / np.abs(b).max()) <= 1e-5, name
    refs = oracle_gradients(g, w.cams, oracle_params(Pm, 320.0), upix, vals.astype(np.float64))
    check_gradients(gm, refs, "training record grads + recomputed state")


@pytest.mark.parametrize("tile", [(8, 8), (32, 8)])
def test_tile_lists_longer_than_the_lds_depth_sort(tile):
    """A dense soup of 30,000 small tets: tiles with over 10,000 entries, more
    than the per-tile depth sort holds in LDS (4096), so their runs are merged
    in HBM (two merge rounds).  Tiling bit-exact, image and gradients against
    the oracle."""
    import torch
    rng = np.random.default_rng(71)
    K = 30000
    centres = rng.normal(scale=0.04, size=(K, 1, 3))
    verts = (centres + rng.normal(scale=0.04, size=(K, 4, 3))).reshape(-1, 3).astype(np.float32)
    tets = np.arange(4 * K, dtype=np.int32).reshape(K, 4)
    sdf = rng.uniform(-0.03, 0.02, size=4 * K).astype(np.float32)
    colors = rng.uniform(0.0, 1.0, size=(4 * K, 3)).astype(np.float32)
    s = 40.0
    sc = synth.Scene(verts, tets, sdf, colors, s, "dense soup")
    cam = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, 64, 64, (0.1, 0.2, 0.3))[None]
    P = _params("default", tile)
    r, plan, imgs = gpu_forward(sc, cam, P)
    d, tets_sorted = gpu_tiling(r, plan)
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, s)
    ref = oracle.binning(g, cam, op)
    lens = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    print(f"soup {tile}: E={ref['E']}, longest list {lens.max()}, lists over 4096: {(lens > 4096).sum()}")
    assert lens.max() > 3 * 4096
    assert d["entries"] == ref["E"]
    assert np.array_equal(d["tile_keys"], ref["tile"].astype(np.uint32))
    assert np.array_equal(tets_sorted, ref["tet"])
    assert np.array_equal(d["ranges"].astype(np.int64), ref["ranges"].astype(np.int64))
    err, n_ex, n = compare_images(imgs, g, cam, op, s)
    assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n))
    dout = rng.normal(size=(8, 64, 64)).astype(np.float32)
    (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
    torch.cuda.synchronize()
    refs = oracle_gradients(g, cam, op, oracle.all_pixels(cam), dout.reshape(8, -1).T.copy())
    check_gradients((dv, ds, dc), refs, f"soup {tile}")
