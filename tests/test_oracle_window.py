"""Pins of the oracle's per-pixel resort window (Sec. 3.3): a window at
least as long as the pixel's candidate list gives the candidates sorted by
their own entry depth (checked with numpy's stable sort of the window-off
trace); a two-tet scene whose per-tile order (mean depth) is the reverse of
its per-pixel order blends in closed form in each order; window 0 is the
plain path; and the windowed reverse mode agrees with forward-mode dual
numbers and central differences."""
import math

import numpy as np
import pytest

import oracle
import synth

EXACT = dict(oracle.EXACT)


def _hot_pixels(g, cams, P, n, seed):
    out = oracle.render(g, cams, P)
    pix = oracle.all_pixels(cams)
    hot = pix[out[:, 3] > 0.05]
    return hot[np.random.default_rng(seed).choice(len(hot), n, replace=False)]


@pytest.mark.parametrize("s", [20.0, 100.0])
def test_long_window_is_the_per_pixel_depth_order(s):
    w = synth.tiny(s=s)
    g = oracle.Geometry.of(w.scenes[0])
    P0 = oracle.params_array(s, **EXACT)
    Pw = oracle.params_array(s, **dict(EXACT, window=4096))
    for (v, i, j) in _hot_pixels(g, w.cams, P0, 40, 1):
        t0 = oracle.pixel_trace(g, w.cams, P0, int(v), int(i), int(j))
        tw = oracle.pixel_trace(g, w.cams, Pw, int(v), int(i), int(j))
        order = np.argsort(t0["zin"], kind="stable")
        assert np.array_equal(tw["tet"], t0["tet"][order])
        assert np.all(np.diff(tw["zin"]) >= 0)


def _two_tets():
    # camera on +x at distance 5 looking at the origin: depth = 5 - x
    cam = synth.orbit_camera(0.0, 0.0, 5.0, 50.0, 32, 32, bg=(0.1, 0.2, 0.3))[None]
    verts = np.array([
        [3.0, -1.0, -1.0], [3.0, 1.0, -1.0], [3.0, 0.0, 1.5], [1.0, 0.0, 0.0],     # A: depths 2,2,2,4 (mean 2.5)
        [2.8, -0.3, -0.3], [2.8, 0.3, -0.3], [2.8, 0.0, 0.4], [2.7, 0.0, 0.0],     # B: 2.2,2.2,2.2,2.3 (mean 2.225)
    ])
    tets = np.array([[0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    sdf = verts[:, 0] - 2.0
    colors = np.array([[1, 0, 0]] * 4 + [[0, 1, 0]] * 4, np.float64)
    return oracle.Geometry(verts, tets, sdf, colors), cam


@pytest.mark.parametrize("window", [0, 1, 3])
def test_two_tets_blend_in_the_order_the_window_gives(window):
    g, cam = _two_tets()
    s = 5.0
    P = oracle.params_array(s, **dict(EXACT, window=window))
    i = j = 16
    tr = oracle.pixel_trace(g, cam, P, 0, i, j)
    assert sorted(tr["tet"].tolist()) == [0, 1]
    # tile order is B (mean depth 2.225) then A (2.5); the pixel enters A at depth 2 and B at 2.2
    expect = [1, 0] if window == 0 else [0, 1]
    assert tr["tet"].tolist() == expect
    a = dict(zip(tr["tet"].tolist(), tr["alpha"].tolist()))
    c = {0: np.array([1.0, 0, 0]), 1: np.array([0, 1.0, 0])}
    first, second = expect
    rgb = a[first] * c[first] + (1 - a[first]) * a[second] * c[second] + \
        (1 - a[first]) * (1 - a[second]) * cam[0, 19:22].astype(np.float64)
    out = oracle.render(g, cam, P, np.array([[0, i, j]], np.int32))[0]
    np.testing.assert_allclose(out[:3], rgb, rtol=1e-12, atol=1e-14)
    assert out[3] == pytest.approx(1 - (1 - a[0]) * (1 - a[1]), rel=1e-12)
    # entry depths at the pixel: 2 for A, 2.2 for B (flat entry faces facing the camera)
    z = dict(zip(tr["tet"].tolist(), tr["zin"].tolist()))
    assert z[0] == pytest.approx(2.0, rel=1e-12) and z[1] == pytest.approx(2.2, rel=1e-12)


def test_window_zero_is_the_plain_path():
    w = synth.tiny(s=20.0)
    g = oracle.Geometry.of(w.scenes[0])
    a = oracle.render(g, w.cams, oracle.params_array(20.0))
    b = oracle.render(g, w.cams, oracle.params_array(20.0, window=0))
    assert np.array_equal(a, b)


def test_windowed_reverse_mode_matches_duals_and_differences():
    w = synth.tiny(s=20.0, bg=(0.3, 0.1, 0.2))
    g = oracle.Geometry.of(w.scenes[0])
    P = oracle.params_array(20.0, **dict(EXACT, window=3))
    pix = oracle.all_pixels(w.cams)
    rng = np.random.default_rng(41)
    wout = rng.normal(size=(pix.shape[0], 8))
    dv, ds, dc = oracle.backward(g, w.cams, P, pix, wout)
    tv, ts, tc = rng.normal(size=(g.V, 3)), rng.normal(size=g.V), rng.normal(size=(g.V, 3))
    _, tout = oracle.render_dual(g, w.cams, P, pix, tv, ts, tc)
    assert float((wout * tout).sum()) == pytest.approx(float((dv * tv).sum() + (ds * ts).sum() + (dc * tc).sum()),
                                                      rel=1e-10)
    hot = _hot_pixels(g, w.cams, P, 10, 3)
    verts = sorted({int(x) for (v, i, j) in hot
                    for k in oracle.pixel_trace(g, w.cams, P, int(v), int(i), int(j))["tet"][:2]
                    for x in g.tets[k]})[:10]

    def loss(gg):
        return float((oracle.render(gg, w.cams, P, pix) * wout).sum())

    for vi in verts:
        gp = oracle.Geometry(g.verts, g.tets, g.sdf.copy(), g.colors)
        gm = oracle.Geometry(g.verts, g.tets, g.sdf.copy(), g.colors)
        gp.sdf[vi] += 1e-6
        gm.sdf[vi] -= 1e-6
        fd = (loss(gp) - loss(gm)) / 2e-6
        assert fd == pytest.approx(ds[vi], rel=2e-4, abs=2e-4 * (abs(ds[vi]) + 1e-2))
