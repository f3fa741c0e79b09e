"""GPU parity of the per-pixel resort window (Sec. 3.3) against the oracle's
window (same candidate order, same buffer rule, same thresholds): images
within 1e-5 max-abs of the float32 oracle, gradients within the gradient bar
of tests/gpu_helpers.py; a two-tet scene whose per-tile order is the reverse
of its per-pixel order blends in the closed form of each order; the number
of waves per tile does not change the result."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import IMG_TOL, check_gradients, oracle_gradients, compare_images, gpu_forward, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _params(mode, window, **kw):
    from paper_2406_01579_amd import Params
    base = Params.exact if mode == "exact" else Params
    return base(tile_w=8, tile_h=8, window=window, **kw)


@pytest.mark.parametrize("window", [1, 3, 5, 8])
@pytest.mark.parametrize("s", [20.0, 100.0])
@pytest.mark.parametrize("mode", ["exact", "default"])
def test_tiny_window_images(mode, s, window):
    w = synth.tiny(s=s, bg=(0.1, 0.2, 0.3))
    sc = w.scenes[0]
    P = _params(mode, window)
    _, _, imgs = gpu_forward(sc, w.cams, P)
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, s)
    err32, n_ex, n = compare_images(imgs, g, w.cams, op, s)
    err64 = np.abs(imgs[0] - oracle.render_images(g, w.cams, op, prec=64)[0]).reshape(8, -1).max(1)
    print(f"window {window} {mode} s={s}: max-abs vs f32 {err32:.3e} (excluded {n_ex}/{n}); vs f64 {err64.max():.3e}")
    assert err32 <= IMG_TOL
    assert n_ex <= max(1, int(1e-4 * n))


def test_window_changes_the_image():
    """The window does reorder blends on the tiny grid (otherwise the tests
    above would not test it)."""
    w = synth.tiny(s=100.0, bg=(0.1, 0.2, 0.3))
    _, _, a = gpu_forward(w.scenes[0], w.cams, _params("default", 0))
    _, _, b = gpu_forward(w.scenes[0], w.cams, _params("default", 5))
    diff = np.abs(a[0] - b[0]).max(axis=0)
    print(f"pixels changed by the window: {(diff > 1e-6).sum()}, max {diff.max():.3e}")
    assert (diff > 1e-6).sum() > 0


@pytest.mark.parametrize("window", [1, 5])
@pytest.mark.parametrize("s", [20.0, 100.0])
@pytest.mark.parametrize("mode", ["exact", "default"])
def test_tiny_window_gradients(mode, s, window):
    import torch
    w = synth.tiny(s=s, bg=(0.3, 0.1, 0.2))
    sc = w.scenes[0]
    P = _params(mode, window)
    r, plan, _ = gpu_forward(sc, w.cams, P)
    dout = np.random.default_rng(5).normal(size=(8, 64, 64)).astype(np.float32)
    (dv, ds, dc), = r.backward(plan, [torch.from_numpy(dout).cuda()])
    torch.cuda.synchronize()
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, s)
    pix = oracle.all_pixels(w.cams)
    dflat = dout.reshape(8, -1).T.copy()
    refs = oracle_gradients(g, w.cams, op, pix, dflat)
    check_gradients((dv, ds, dc), refs, f"window {window} {mode} s={s}")


@pytest.mark.parametrize("waves", [1, 2, 8])
def test_waves_per_tile_do_not_change_window_results(waves):
    import torch
    w = synth.tiny(s=100.0, bg=(0.3, 0.3, 0.3))
    sc = w.scenes[0]
    dout = torch.from_numpy(np.random.default_rng(8).normal(size=(8, 64, 64)).astype(np.float32)).cuda()
    res = []
    for wv in (4, waves):
        r, plan, imgs = gpu_forward(sc, w.cams, _params("default", 5, waves=wv))
        grads = [t.cpu().numpy() for t in r.backward(plan, [dout])[0]]
        res.append((imgs[0], grads))
    assert np.array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(b).max())


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_window_gradients_repeat_bitwise(waves):
    """The resort-window backward with several waves per tile gives the same
    gradients, bit for bit, on repeats of the same input (fixed-order sums):
    each pixel's blend records, the entries' blend masks and pair places pass
    between waves only across the kernel's barriers, and the masks, set by
    atomics, are read from L2."""
    import torch
    w = synth.training(s=320.0, R=16, size=96, views=2)
    sc = w.scenes[0]
    P = _params("default", 5, waves=waves, deterministic=True)
    gen = np.random.default_rng(12)
    douts = [torch.from_numpy(gen.normal(size=(8, 96, 96)).astype(np.float32)).cuda() for _ in range(2)]
    r, plan, _ = gpu_forward(sc, w.cams, P)
    ref = [t.cpu().numpy() for t in r.backward(plan, douts)[0]]
    assert max(np.abs(t).max() for t in ref) > 0
    for _ in range(8):
        r, plan, _ = gpu_forward(sc, w.cams, P)
        got = [t.cpu().numpy() for t in r.backward(plan, douts)[0]]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def _two_tets():
    # camera on +x at distance 5 looking at the origin: depth = 5 - x
    cam = synth.orbit_camera(0.0, 0.0, 5.0, 50.0, 32, 32, bg=(0.1, 0.2, 0.3))[None]
    verts = np.array([
        [3.0, -1.0, -1.0], [3.0, 1.0, -1.0], [3.0, 0.0, 1.5], [1.0, 0.0, 0.0],     # A: depths 2,2,2,4 (mean 2.5)
        [2.8, -0.3, -0.3], [2.8, 0.3, -0.3], [2.8, 0.0, 0.4], [2.7, 0.0, 0.0],     # B: 2.2,2.2,2.2,2.3 (mean 2.225)
    ], np.float32)
    tets = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    sdf = (verts[:, 0] - 2.0).astype(np.float32)
    colors = np.array([[1, 0, 0]] * 4 + [[0, 1, 0]] * 4, np.float32)
    return synth.Scene(verts, tets, sdf, colors, 5.0), cam


@pytest.mark.parametrize("window", [0, 1, 3])
def test_two_tets_blend_in_the_order_the_window_gives(window):
    """Tile order is B (mean depth 2.225) then A (2.5); the centre pixel's ray
    enters A at depth 2 and B at 2.2, so any window blends A first."""
    sc, cam = _two_tets()
    P = _params("exact", window)
    _, _, imgs = gpu_forward(sc, cam, P)
    g = oracle.Geometry.of(sc)
    op = oracle_params(P, 5.0)
    tr = oracle.pixel_trace(g, cam, op, 0, 16, 16)
    a = dict(zip(tr["tet"].tolist(), tr["alpha"].tolist()))
    first, second = (1, 0) if window == 0 else (0, 1)
    col = {0: np.array([1.0, 0, 0]), 1: np.array([0, 1.0, 0])}
    rgb = a[first] * col[first] + (1 - a[first]) * a[second] * col[second] + \
        (1 - a[first]) * (1 - a[second]) * np.array([0.1, 0.2, 0.3])
    got = imgs[0][:3, 16, 16].astype(np.float64)
    print(f"window {window}: got {got}, closed form {rgb}")
    np.testing.assert_allclose(got, rgb, atol=2e-6)
    err, n_ex, n = compare_images(imgs, g, cam, op, 5.0)
    assert err <= IMG_TOL and n_ex == 0


@pytest.mark.parametrize("size", [(50, 37), (130, 9)])
def test_window_ragged_image_sizes(size):
    s = 100.0
    w = synth.tiny(s=s, bg=(0.2, 0.5, 0.1))
    Wd, Hd = size
    cam = synth.orbit_camera(0.7, 0.35, 2.5, 50.0, Wd, Hd, bg=(0.2, 0.5, 0.1))[None]
    cam[0, 17] = Hd / 2.0
    P = _params("default", 5)
    _, _, imgs = gpu_forward(w.scenes[0], cam, P)
    err, n_ex, n = compare_images(imgs, oracle.Geometry.of(w.scenes[0]), cam, oracle_params(P, s), s)
    assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n)), size


def test_window_empty_scene():
    import torch
    w = synth.tiny(s=20.0, bg=(0.25, 0.5, 0.75))
    sc = w.scenes[0]
    empty = synth.Scene(sc.verts, sc.tets, np.full_like(sc.sdf, 2.0), sc.colors, 20.0)
    r, plan, imgs = gpu_forward(empty, w.cams, _params("default", 5))
    bg = np.array([0.25, 0.5, 0.75], np.float32)
    assert np.array_equal(imgs[0][0:3], np.broadcast_to(bg[:, None, None], (3, 64, 64)))
    assert np.all(imgs[0][3:] == 0)
    (dv, ds, dc), = r.backward(plan, [torch.ones(8, 64, 64, device="cuda")])
    assert float(dv.abs().max()) == 0 and float(ds.abs().max()) == 0 and float(dc.abs().max()) == 0


# ---------------------------------------------------------------------------
# training-shaped workload at full size (64^3 grid, 4 views 512^2, s = 320),
# the paper's window N_w = 5: sampled pixels and a sparse upstream gradient
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def training():
    w = synth.training(s=320.0)
    return w, oracle.Geometry.of(w.scenes[0])


def test_training_window_sampled_pixels(training):
    w, g = training
    P = _params("default", 5)
    _, _, imgs = gpu_forward(w.scenes[0], w.cams, P)
    rng = np.random.default_rng(1)
    pix = np.stack([rng.integers(0, 4, 2000), rng.integers(0, 512, 2000), rng.integers(0, 512, 2000)], 1)
    cov = np.argwhere(np.stack(imgs)[:, 3] > 0.01)
    pick = cov[np.random.default_rng(2).choice(len(cov), 2000, replace=False)]
    pix = np.ascontiguousarray(np.concatenate([pix, pick[:, [0, 2, 1]]], 0), dtype=np.int32)
    op = oracle_params(P, 320.0)
    err, n_ex, n = compare_images(imgs, g, w.cams, op, 320.0, pix=pix)
    print(f"training window 5: sampled max-abs vs f32 {err:.3e} (excluded {n_ex}/{n})")
    assert err <= IMG_TOL and n_ex <= max(1, int(1e-4 * n))


def test_training_window_gradients_of_sparse_upstream(training):
    import torch
    w, g = training
    P = _params("default", 5)
    r, plan, imgs = gpu_forward(w.scenes[0], w.cams, P)
    cov = np.argwhere(np.stack(imgs)[:, 3] > 0.01)
    pick = cov[np.random.default_rng(3).choice(len(cov), 2000, replace=False)]
    pix = np.ascontiguousarray(pick[:, [0, 2, 1]], dtype=np.int32)
    vals = np.random.default_rng(4).normal(size=(pix.shape[0], 8)).astype(np.float32)
    douts = [np.zeros((8, 512, 512), np.float32) for _ in range(4)]
    for (v, i, j), x in zip(pix, vals):
        douts[v][:, j, i] += x
    key = pix[:, 0] * 512 * 512 + pix[:, 2] * 512 + pix[:, 1]
    _, first = np.unique(key, return_index=True)
    upix = pix[first]
    dflat = np.stack([douts[v][:, j, i] for (v, i, j) in upix], 0).astype(np.float64)
    grads, = r.backward(plan, [torch.from_numpy(d).cuda() for d in douts])
    torch.cuda.synchronize()
    op = oracle_params(P, 320.0)
    refs = oracle_gradients(g, w.cams, op, upix, dflat)
    check_gradients(grads, refs, "training window 5 sparse-upstream")


# ---------------------------------------------------------------------------
# sorting error (Sec. 3.3): images under the per-tile order and under windows
# of several sizes, against the exact per-pixel order (the oracle's window
# longer than any pixel's list), on the training-shaped grid at two
# resolutions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("R", [64, 128])
def test_window_sort_error_against_exact_per_pixel_order(R):
    w = synth.training(s=320.0, R=R)
    g = oracle.Geometry.of(w.scenes[0])
    _, _, base = gpu_forward(w.scenes[0], w.cams, _params("default", 0))
    cov = np.argwhere(np.stack(base)[:, 3] > 0.01)
    pick = cov[np.random.default_rng(7).choice(len(cov), 3000, replace=False)]
    pix = np.ascontiguousarray(pick[:, [0, 2, 1]], dtype=np.int32)
    exact = oracle.render(g, w.cams, oracle.params_array(320.0, tile_w=8, tile_h=8, window=4096), pix, prec=32)
    stats = {}
    for nw in (0, 1, 3, 5, 8):
        _, _, imgs = gpu_forward(w.scenes[0], w.cams, _params("default", nw))
        got = np.stack([imgs[v][:, j, i] for (v, i, j) in pix], 0)
        err = np.abs(got[:, :3] - exact[:, :3]).max(axis=1)
        stats[nw] = (float((err > 1e-3).mean()), float(err.mean()), float(err.max()))
        print(f"R={R} window {nw}: pixels off the exact order's colour by >1e-3: {100 * stats[nw][0]:.2f}%, "
              f"mean {stats[nw][1]:.2e}, max {stats[nw][2]:.3f}")
    assert stats[8][0] <= stats[0][0] and stats[5][1] <= stats[0][1]
