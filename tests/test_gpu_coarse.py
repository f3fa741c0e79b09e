"""Coarse-to-fine pre-filtering on the GPU against the oracle: the kept box
and count bit-exact (up to tets whose alpha_max lies within float32 rounding
of T_f), NaN box for an empty kept set, and the whole two-pass rebuild equal
to the oracle's composition of the same steps."""
import numpy as np
import pytest

import synth
from oracle import coarse as ocoarse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _scene(name):
    if name == "tiny":
        sc = synth.tiny().scenes[0]
    elif name == "training":
        sc = synth.training().scenes[0]
    else:
        sc = synth.batched().scenes[0]
    return sc


@pytest.mark.parametrize("name", ["tiny", "training", "batched"])
def test_bounds_match_oracle(name):
    import torch
    from paper_2406_01579_amd import SceneT
    from paper_2406_01579_amd.coarse import prefilter_bounds
    sc = _scene(name)
    b, k = prefilter_bounds(SceneT.from_numpy(sc))
    got, kept = b.cpu().numpy(), int(k.item())
    lo, hi, n = ocoarse.kept_bounds(sc.verts, sc.tets, sc.sdf, sc.s)
    print(f"{name}: kept {kept} vs {n}; box {got}")
    assert abs(kept - n) <= max(2, n // 100000)
    assert np.array_equal(got, np.concatenate([lo, hi]))
    sc2 = SceneT.from_numpy(sc)
    sc2.sdf.fill_(5.0)
    b2, k2 = prefilter_bounds(sc2)
    assert int(k2.item()) == 0 and np.all(np.isnan(b2.cpu().numpy()))


def test_two_pass_rebuild_matches_oracle():
    import torch
    from paper_2406_01579_amd.coarse import coarse_to_fine
    R, s = 32, 320.0
    c, r = np.array([0.25, -0.15, 0.1], np.float32), 0.35

    def sdf_fn(v):
        return torch.linalg.norm(v - torch.as_tensor(c, device=v.device), dim=1) - r

    v2, t2, f2, info = coarse_to_fine(sdf_fn, R, s)
    # oracle: the first pass on the same grid and SDF values, then the rebuilt cube
    verts1, tets1 = synth.kuhn_grid(R)
    v1 = ocoarse.grid_vertices(np.full(3, -1.0, np.float32), np.float32(2.0 / R), R)
    f1 = sdf_fn(torch.from_numpy(v1).cuda()).cpu().numpy()
    lo, hi, n = ocoarse.kept_bounds(v1, tets1, f1, s)
    assert info["pass1_kept"] == n and np.array_equal(info["pass1_box"], np.concatenate([lo, hi]))
    low, h = ocoarse.resized_cube(lo, hi, R, np.float32(2.0 / R))
    assert np.array_equal(v2.cpu().numpy(), ocoarse.grid_vertices(low, h, R))
    assert np.array_equal(t2.cpu().numpy(), tets1.astype(np.int32))
    # the rebuilt grid is finer around the surface and still holds all of it
    assert float(h) < 2.0 / R
    lo2, hi2, n2 = ocoarse.kept_bounds(v2.cpu().numpy(), tets1, f2.cpu().numpy(), s)
    assert n2 > n and np.all(lo2 >= low) and np.all(hi2 <= low + float(h) * R)
