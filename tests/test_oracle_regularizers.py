"""Pins of the regulariser oracle (Sec. 4.2, App. A.3) against facts fixed
outside it: the edge count of the Kuhn cube triangulation, the 4x4 system of
App. A.3 as an independent route to g, closed forms for a linear SDF and for
a two-tet mesh with orthogonal normals, exclusion of a flat tet, scale
invariance of the normal term, and central finite differences."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import regularizers as R


@pytest.mark.parametrize("n", [1, 2, 3])
def test_kuhn_grid_edge_count(n):
    # axis edges + one diagonal per square face + one body diagonal per cube
    _, tets = synth.kuhn_grid(n)
    assert len(R.mesh_edges(tets)) == 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3


def test_gradient_matches_the_4x4_system():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(50, 4, 3))
    f = rng.normal(size=(50, 4))
    verts = torch.tensor(x.reshape(-1, 3))
    tets = np.arange(200).reshape(50, 4)
    g, ok = R.tet_gradients(verts, torch.as_tensor(tets), torch.tensor(f.ravel()))
    for k in range(50):
        A = np.concatenate([x[k], np.ones((4, 1))], 1)        # [x_a 1] [g; b] = f_a
        gb = np.linalg.solve(A, f[k])
        np.testing.assert_allclose(g[k].numpy(), gb[:3], rtol=1e-9, atol=1e-9)
    assert bool(ok.all())


def test_linear_sdf_closed_forms():
    verts, tets = synth.kuhn_grid(3)
    rng = np.random.default_rng(1)
    verts = verts + rng.uniform(-0.05, 0.05, verts.shape)
    a = np.array([0.3, -1.2, 0.7])
    sdf = verts @ a + 0.1
    le, ln, dv, df = R.losses_and_grads(verts, tets, sdf)
    assert le == pytest.approx(len(tets) * (np.linalg.norm(a) - 1.0) ** 2, rel=1e-10)
    assert abs(ln) < 1e-10
    a1 = a / np.linalg.norm(a)
    le1, ln1, _, _ = R.losses_and_grads(verts, tets, verts @ a1)
    assert abs(le1) < 1e-18 and abs(ln1) < 1e-10


def test_two_tets_with_orthogonal_normals():
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4]])
    sdf = np.array([0.0, 1.0, 0.0, 1.0, 1.0])      # g_A = (1,0,1), g_B = (1,0,-1)
    le, ln, _, _ = R.losses_and_grads(verts, tets, sdf)
    assert le == pytest.approx(2 * (math.sqrt(2) - 1) ** 2, rel=1e-12)
    assert ln == pytest.approx(6 * (1 - 1 / math.sqrt(2)), rel=1e-12)
    # each term on its own
    le2, ln2, _, _ = R.losses_and_grads(verts, tets[:1], sdf)
    assert le2 == pytest.approx((math.sqrt(2) - 1) ** 2, rel=1e-12) and abs(ln2) < 1e-14


def test_flat_tet_is_left_out():
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]], np.float64)
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4]])   # the second is flat (z = 0)
    sdf = np.array([0.0, 2.0, 0.0, 0.0, 5.0])
    le, _, _, _ = R.losses_and_grads(verts, tets, sdf)
    assert le == pytest.approx((2.0 - 1.0) ** 2, rel=1e-12)


def test_normal_term_is_scale_invariant():
    w = synth.tiny()
    sc = w.scenes[0]
    _, ln, _, _ = R.losses_and_grads(sc.verts, sc.tets, sc.sdf)
    _, ln3, _, _ = R.losses_and_grads(sc.verts, sc.tets, 3.0 * sc.sdf.astype(np.float64))
    assert ln > 1e-3 and ln3 == pytest.approx(ln, rel=1e-10)


def test_gradients_match_central_differences():
    verts, tets = synth.kuhn_grid(2)
    rng = np.random.default_rng(2)
    verts = verts + rng.uniform(-0.08, 0.08, verts.shape)
    sdf = np.linalg.norm(verts, axis=1) - 0.6 + rng.normal(0, 0.05, len(verts))
    w_eik, w_nc = 0.7, 1.3
    _, _, dv, df = R.losses_and_grads(verts, tets, sdf, w_eik, w_nc)

    def total(v, f):
        le, ln, _, _ = R.losses_and_grads(v, tets, f, w_eik, w_nc)
        return w_eik * le + w_nc * ln

    h = 1e-6
    for i in rng.choice(len(verts), 8, replace=False):
        e = np.zeros_like(sdf)
        e[i] = h
        fd = (total(verts, sdf + e) - total(verts, sdf - e)) / (2 * h)
        assert fd == pytest.approx(df[i], rel=1e-5, abs=1e-7)
        for m in range(3):
            E = np.zeros_like(verts)
            E[i, m] = h
            fd = (total(verts + E, sdf) - total(verts - E, sdf)) / (2 * h)
            assert fd == pytest.approx(dv[i, m], rel=1e-5, abs=1e-7)
