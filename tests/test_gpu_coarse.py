"""Coarse-to-fine pre-filtering on the GPU (App. B) against the oracle, every
step through the C ABI: the kept box and count (bit-exact up to tets whose
alpha_max lies within float32 rounding of T_f; NaN box for an empty kept
set), the refitted second-pass cube and the rebuilt grid bit-exact, and the
whole two-pass rebuild equal to the oracle's composition of the same steps."""
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


@pytest.mark.parametrize("R", [1, 5, 16, 33])
def test_cube_grid_matches_oracle_and_generator(R):
    import torch
    from paper_2406_01579_amd.coarse import cube_grid
    rng = np.random.default_rng(R)
    low = rng.uniform(-1, 0.5, 3).astype(np.float32)
    h = np.float32(rng.uniform(0.01, 0.3))
    cube = torch.tensor(np.concatenate([low, [h]]), dtype=torch.float32, device="cuda")
    v, t = cube_grid(R, cube)
    _, t_ref = synth.kuhn_grid(R)
    assert np.array_equal(t.cpu().numpy(), t_ref.astype(np.int32))
    assert np.array_equal(v.cpu().numpy(), ocoarse.grid_vertices(low, h, R))
    v2, t2 = cube_grid(R, cube, with_tets=False)
    assert t2 is None and np.array_equal(v2.cpu().numpy(), v.cpu().numpy())


def test_refit_cube_matches_oracle():
    """Random boxes (including degenerate, flat and off-centre ones): the
    device cube equals the oracle's bit for bit; a NaN box keeps the cube."""
    import torch
    from paper_2406_01579_amd.coarse import refit_cube
    rng = np.random.default_rng(17)
    for trial in range(200):
        R = int(rng.choice([8, 16, 32, 64, 128, 100]))
        old_h = np.float32(2.0 / R) if trial % 3 else np.float32(rng.uniform(0.001, 0.2))
        lo = rng.uniform(-1, 1, 3).astype(np.float32)
        ext = rng.uniform(0, 1.5, 3).astype(np.float32)
        if trial % 7 == 0:
            ext[rng.integers(0, 3)] = 0.0
        if trial % 11 == 0:
            ext[:] = 0.0
        hi = (lo + ext).astype(np.float32)
        cube_in = np.array([-1, -1, -1, old_h], np.float32)
        box = torch.tensor(np.concatenate([lo, hi]), device="cuda")
        got = refit_cube(box, torch.tensor(cube_in, device="cuda"), R).cpu().numpy()
        low, h = ocoarse.resized_cube(lo, hi, R, old_h)
        assert np.array_equal(got[:3], low) and got[3] == h, (trial, got, low, h)
    nan_box = torch.full((6,), float("nan"), device="cuda")
    cube_in = torch.tensor([0.25, -0.5, 0.125, 0.0625], device="cuda")
    assert torch.equal(refit_cube(nan_box, cube_in, 16), cube_in)


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
    assert int(info["pass1_kept"].item()) == n
    assert np.array_equal(info["pass1_box"].cpu().numpy(), np.concatenate([lo, hi]))
    low, h = ocoarse.resized_cube(lo, hi, R, np.float32(2.0 / R))
    cube = info["cube"].cpu().numpy()
    assert np.array_equal(cube[:3], low) and cube[3] == h
    assert np.array_equal(v2.cpu().numpy(), ocoarse.grid_vertices(low, h, R))
    assert np.array_equal(t2.cpu().numpy(), tets1.astype(np.int32))
    # the rebuilt grid is finer around the surface and still holds all of it
    assert float(h) < 2.0 / R
    lo2, hi2, n2 = ocoarse.kept_bounds(v2.cpu().numpy(), tets1, f2.cpu().numpy(), s)
    assert n2 > n and np.all(lo2 >= low) and np.all(hi2 <= low + float(h) * R)


def test_two_pass_with_nothing_kept_keeps_the_grid():
    import torch
    from paper_2406_01579_amd.coarse import coarse_to_fine
    R = 8
    v2, t2, f2, info = coarse_to_fine(lambda v: torch.full((v.shape[0],), 3.0, device=v.device), R, 320.0)
    assert int(info["pass1_kept"].item()) == 0
    assert torch.equal(info["cube"], info["cube1"])
    assert np.array_equal(v2.cpu().numpy(), ocoarse.grid_vertices(np.full(3, -1.0, np.float32),
                                                                  np.float32(2.0 / R), R))
