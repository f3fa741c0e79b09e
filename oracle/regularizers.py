"""Oracle of the two geometry regularisers (Sec. 4.2), float64 on the CPU.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never does.

Definitions (readings listed with the rest of the paper's readings):
  * per-tet SDF gradient g_k: the gradient of the linear interpolant of the
    four vertex SDF values over the tet (App. A.3), i.e. the solution of
    E g = df with E's rows x_a - x_0 and df_a = f_a - f_0 (a = 1..3);
    a tet with det E = 0 has no gradient and is left out of both terms;
  * eikonal term: L_eik = sum over tets of (|g_k| - 1)^2;
  * tet normal n_k = g_k / |g_k| (0 if g_k = 0); vertex normal m_v = the sum
    of the normals of the tets that contain v ("projected onto vertices");
  * normal-consistency term: L_nc = sum over the undirected edges (a, b) of
    the tet mesh, each counted once, of 1 - cos(m_a, m_b); an edge with a
    zero vertex normal at either end is left out.
Both terms run over every tet of the grid.  Gradients with respect to the
vertex positions and the SDF values are taken by reverse-mode automatic
differentiation of these definitions (torch, float64).
"""
from __future__ import annotations

import numpy as np
import torch


def mesh_edges(tets) -> np.ndarray:
    """Unique undirected edges (a < b) of a tet mesh, sorted by (a, b)."""
    t = np.asarray(tets, np.int64)
    pairs = np.concatenate([t[:, [i, j]] for i, j in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))], 0)
    pairs.sort(axis=1)
    return np.unique(pairs, axis=0)


def tet_gradients(verts, tets, sdf):
    """g [K,3] and the mask of non-degenerate tets (App. A.3)."""
    x = verts[tets]                              # [K,4,3]
    f = sdf[tets]                                # [K,4]
    E = x[:, 1:, :] - x[:, :1, :]                # [K,3,3]
    df = (f[:, 1:] - f[:, :1]).unsqueeze(-1)     # [K,3,1]
    det = torch.linalg.det(E)
    ok = det != 0
    g = torch.zeros(tets.shape[0], 3, dtype=verts.dtype)
    if bool(ok.any()):
        g = g.index_put((ok.nonzero().squeeze(1),), torch.linalg.solve(E[ok], df[ok]).squeeze(-1))
    return g, ok


def losses(verts, tets, sdf, edges=None):
    """(L_eik, L_nc) as float64 tensors (Sec. 4.2)."""
    tets = torch.as_tensor(np.asarray(tets, np.int64))
    if edges is None:
        edges = mesh_edges(tets.numpy())
    edges = torch.as_tensor(np.asarray(edges, np.int64))
    g, ok = tet_gradients(verts, tets, sdf)
    gn = torch.linalg.norm(g[ok], dim=1)
    l_eik = ((gn - 1.0) ** 2).sum()
    n = torch.zeros_like(g)
    nz = ok.clone()
    nz[ok] = gn > 0
    n[nz] = g[nz] / torch.linalg.norm(g[nz], dim=1, keepdim=True)
    m = torch.zeros_like(verts).index_add(0, tets.reshape(-1), n.repeat_interleave(4, dim=0))
    ma, mb = m[edges[:, 0]], m[edges[:, 1]]
    na, nb = torch.linalg.norm(ma, dim=1), torch.linalg.norm(mb, dim=1)
    use = (na > 0) & (nb > 0)
    cos = (ma[use] * mb[use]).sum(1) / (na[use] * nb[use])
    l_nc = (1.0 - cos).sum()
    return l_eik, l_nc


def losses_and_grads(verts, tets, sdf, w_eik=1.0, w_nc=1.0, edges=None):
    """L_eik, L_nc and the gradients of w_eik*L_eik + w_nc*L_nc with respect
    to the vertex positions [V,3] and the SDF values [V] (numpy float64)."""
    v = torch.tensor(np.asarray(verts, np.float64), requires_grad=True)
    f = torch.tensor(np.asarray(sdf, np.float64), requires_grad=True)
    le, ln = losses(v, tets, f, edges)
    total = w_eik * le + w_nc * ln
    dv, df = torch.autograd.grad(total, (v, f), allow_unused=True)
    dv = torch.zeros_like(v) if dv is None else dv
    df = torch.zeros_like(f) if df is None else df
    return le.item(), ln.item(), dv.numpy(), df.numpy()
