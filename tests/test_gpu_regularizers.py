"""Regularisers of Sec. 4.2 on the GPU against the float64 oracle: the edge
list bit-exact (including a mesh with out-of-range indices), both losses to
1e-5 relative, the gradients of a weighted sum normwise to 1e-4, on the tiny
and the training-shaped grids; autograd through the binding."""
import numpy as np
import pytest

import synth
from oracle import regularizers as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a, dt):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda").to(dt).contiguous()


def _scene(name):
    if name == "tiny":
        return synth.tiny().scenes[0]
    if name == "jitter12":
        verts, tets = synth.kuhn_grid(12)
        rng = np.random.default_rng(5)
        verts = verts + rng.uniform(-0.02, 0.02, verts.shape)
        sdf = np.linalg.norm(verts, axis=1) - 0.55 + rng.normal(0, 0.02, len(verts))
        return synth.Scene(verts.astype(np.float32), tets, sdf.astype(np.float32),
                           np.zeros_like(verts, np.float32), 100.0, "jitter12", 12)
    return synth.training(R=32, size=64, views=1).scenes[0]


@pytest.mark.parametrize("name", ["tiny", "jitter12", "training32"])
def test_edges_losses_and_gradients(name):
    import torch
    from paper_2406_01579_amd.regularizers import MeshEdges, _run
    sc = _scene(name)
    V = len(sc.verts)
    v, f, t = _dev(sc.verts, torch.float32), _dev(sc.sdf, torch.float32), _dev(sc.tets, torch.int32)
    me = MeshEdges(t, V)
    ref_edges = R.mesh_edges(sc.tets)
    got = me.edges.cpu().numpy()
    assert np.array_equal(got, ref_edges)
    w = (0.7, 1.3)
    le, ln, dv, df = R.losses_and_grads(sc.verts.astype(np.float64), sc.tets, sc.sdf.astype(np.float64), *w,
                                        edges=ref_edges)
    gdv, gdf = torch.zeros_like(v), torch.zeros_like(f)
    losses = _run(v, f, t, me, torch.tensor(w, device="cuda", dtype=torch.float32), gdv, gdf).cpu().numpy()
    print(f"{name}: L_eik {losses[0]:.9g} vs {le:.9g}, L_nc {losses[1]:.9g} vs {ln:.9g}")
    assert abs(losses[0] - le) <= 1e-5 * abs(le)
    assert abs(losses[1] - ln) <= 1e-5 * abs(ln)
    for got_g, ref in ((gdv.cpu().numpy(), dv), (gdf.cpu().numpy(), df)):
        err = np.abs(got_g - ref).max() / np.abs(ref).max()
        print(f"  grad normwise {err:.2e}")
        assert err <= 1e-4
    # losses alone equal the losses of the gradient run
    l2 = _run(v, f, t, me).cpu().numpy()
    np.testing.assert_allclose(l2, losses, rtol=1e-6)


def test_gradients_are_added_and_autograd_matches():
    import torch
    from paper_2406_01579_amd.regularizers import MeshEdges, _run, regularizers
    sc = _scene("tiny")
    v = _dev(sc.verts, torch.float32).requires_grad_(True)
    f = _dev(sc.sdf, torch.float32).requires_grad_(True)
    t = _dev(sc.tets, torch.int32)
    me = MeshEdges(t, len(sc.verts))
    L = regularizers(v, f, t, me)
    (3.0 * L[0] + 0.5 * L[1]).backward()
    dv0, df0 = torch.zeros_like(v), torch.zeros_like(f)
    w = torch.tensor([3.0, 0.5], device="cuda")
    _run(v.detach(), f.detach(), t, me, w, dv0, df0)
    # float atomics: equal up to summation order, so normwise
    def close(a, b):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()
    close(v.grad, dv0)
    close(f.grad, df0)
    # accumulation: a second call adds the same gradient again
    _run(v.detach(), f.detach(), t, me, w, dv0, df0)
    close(dv0, 2 * v.grad)


def test_out_of_range_tets_are_dropped_and_empty_mesh():
    import torch
    from paper_2406_01579_amd.regularizers import MeshEdges, _run
    sc = _scene("tiny")
    tets = sc.tets.copy()
    bad = np.arange(0, len(tets), 97)
    tets[bad, 2] = len(sc.verts) + 5
    good = np.setdiff1d(np.arange(len(tets)), bad)
    t = _dev(tets, torch.int32)
    me = MeshEdges(t, len(sc.verts))
    assert np.array_equal(me.edges.cpu().numpy(), R.mesh_edges(sc.tets[good]))
    v, f = _dev(sc.verts, torch.float32), _dev(sc.sdf, torch.float32)
    le, ln, _, _ = R.losses_and_grads(sc.verts, sc.tets[good], sc.sdf)
    got = _run(v, f, t, me).cpu().numpy()
    assert abs(got[0] - le) <= 1e-5 * le and abs(got[1] - ln) <= 1e-5 * ln
    e0 = MeshEdges(torch.zeros((0, 4), dtype=torch.int32, device="cuda"), 10)
    assert int(e0.count.item()) == 0
    z = _run(v, f, torch.zeros((0, 4), dtype=torch.int32, device="cuda"), e0).cpu().numpy()
    assert z[0] == 0.0 and z[1] == 0.0
