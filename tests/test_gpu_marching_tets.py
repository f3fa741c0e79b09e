"""Marching Tetrahedra on the GPU against the float64 oracle: triangles
(vertex indices, winding) bit-exact, vertex positions within 2e-6 absolute
(float32 interpolation on coordinates in [-1, 1]), counts exact; a sphere,
the training SDF, a jittered grid with a negatively oriented tet order, and
the capacity and empty cases."""
import numpy as np
import pytest

import synth
from oracle import marching_tets as MT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(name):
    if name == "sphere10":
        verts, tets = synth.kuhn_grid(10)
        sdf = np.linalg.norm(verts, axis=1) - 0.6
    elif name == "training16":
        sc = synth.training(R=16, size=64, views=1).scenes[0]
        verts, tets, sdf = sc.verts, sc.tets, sc.sdf
    else:
        verts, tets = synth.kuhn_grid(9)
        rng = np.random.default_rng(4)
        verts = verts + rng.uniform(-0.03, 0.03, verts.shape)
        tets = tets.copy()
        tets[::3] = tets[::3][:, [0, 2, 1, 3]]            # every third tet negatively oriented
        sdf = np.sin(3 * verts[:, 0]) * np.cos(2 * verts[:, 1]) + verts[:, 2] * 0.5 - 0.1
    return verts.astype(np.float32), np.ascontiguousarray(tets, np.int32), sdf.astype(np.float32)


@pytest.mark.parametrize("name", ["sphere10", "training16", "jitter9"])
def test_mesh_matches_oracle(name):
    import torch
    from paper_2406_01579_amd.mesh import marching_tets
    verts, tets, sdf = _case(name)
    pts, tris, _ = MT.extract(verts.astype(np.float64), tets, sdf.astype(np.float64))
    gv, gt = marching_tets(torch.from_numpy(verts).cuda(), torch.from_numpy(sdf).cuda(),
                           torch.from_numpy(tets).cuda())
    gv, gt = gv.cpu().numpy(), gt.cpu().numpy()
    print(f"{name}: {len(pts)} vertices, {len(tris)} triangles; max |dp| {np.abs(gv - pts).max():.2e}")
    assert gv.shape == pts.shape and gt.shape == tris.shape
    assert np.array_equal(gt, tris)
    assert np.abs(gv - pts).max() <= 2e-6


def test_capacity_shortfall_is_reported_and_empty_grid():
    import torch
    from paper_2406_01579_amd.mesh import marching_tets
    verts, tets, sdf = _case("sphere10")
    v, f, t = (torch.from_numpy(a).cuda() for a in (verts, sdf, tets))
    with pytest.raises(RuntimeError, match="capacities"):
        marching_tets(v, f, t, tri_capacity=10)
    gv, gt = marching_tets(v, torch.ones_like(f), t)
    assert gv.shape[0] == 0 and gt.shape[0] == 0
