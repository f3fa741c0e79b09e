"""Oracle of Marching Tetrahedra mesh extraction (Sec. 4.1, texture stage:
the optimised SDF on the tet grid is turned into a triangle mesh), float64,
CPU.  Test infrastructure only.

Definitions (readings listed with the rest of the paper's readings):
  * a vertex is inside when its SDF value is < 0 (0 counts as outside);
  * every mesh edge (a < b) whose two ends differ in that test carries one
    surface vertex, at the zero of the linear interpolant along the edge,
    p = x_a + t (x_b - x_a) with t = f_a / (f_a - f_b); surface vertices are
    numbered in ascending (a, b) order of their edges;
  * a tet with one or three inside vertices gives one triangle on the three
    crossed edges of the lone vertex, a tet with two gives the two
    triangles of the quad of its four crossed edges; triangles are listed in
    tet order, the two of a quad in a fixed order;
  * triangles face outward (their normal points from the inside vertices to
    the outside ones).  The winding is fixed combinatorially: for the vertex
    order (i, j, k, l) an even permutation of the tet's own order, with i the
    lone vertex (or {i, j} the inside pair), the triangle (e_ij, e_ik, e_il),
    or the quad (e_ik, e_il, e_jl, e_jk) split as (e_ik, e_il, e_jl),
    (e_ik, e_jl, e_jk), faces away from i (from {i, j}) when the tet is
    positively oriented (det[x_1-x_0, x_2-x_0, x_3-x_0] >= 0); it is
    reversed for a negatively oriented tet and for a lone OUTSIDE vertex.
"""
from __future__ import annotations

import numpy as np

from .regularizers import mesh_edges


def _parity(p) -> int:
    p = list(p)
    s = 0
    for a in range(4):
        for b in range(a + 1, 4):
            s += p[a] > p[b]
    return s & 1


def _even(order):
    """The order with its last two entries swapped if needed to be even."""
    o = list(order)
    if _parity(o):
        o[2], o[3] = o[3], o[2]
    return o


def extract(verts, tets, sdf):
    """(vertices [Nv,3] float64, triangles [Nt,3] int64, edge ids of the
    vertices [Nv,2])."""
    verts = np.asarray(verts, np.float64)
    sdf = np.asarray(sdf, np.float64)
    tets = np.asarray(tets, np.int64)
    edges = mesh_edges(tets)
    inside = sdf < 0
    cross = inside[edges[:, 0]] != inside[edges[:, 1]]
    ce = edges[cross]
    fa, fb = sdf[ce[:, 0]], sdf[ce[:, 1]]
    t = fa / (fa - fb)
    pts = verts[ce[:, 0]] + t[:, None] * (verts[ce[:, 1]] - verts[ce[:, 0]])
    vid = {(int(a), int(b)): n for n, (a, b) in enumerate(ce)}

    def e(u, v):
        return vid[(min(u, v), max(u, v))]

    tris = []
    for k in range(tets.shape[0]):
        v = tets[k]
        ins = [int(inside[x]) for x in v]
        c = sum(ins)
        if c in (0, 4):
            continue
        x = verts[v]
        det = np.linalg.det(np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]]))
        flip = det < 0
        if c in (1, 3):
            lone = [q for q in range(4) if ins[q] == (1 if c == 1 else 0)][0]
            o = _even([lone] + [q for q in range(4) if q != lone])
            tri = [e(v[o[0]], v[o[1]]), e(v[o[0]], v[o[2]]), e(v[o[0]], v[o[3]])]
            if flip ^ (c == 3):
                tri = [tri[0], tri[2], tri[1]]
            tris.append(tri)
        else:
            ii = [q for q in range(4) if ins[q]]
            oo = [q for q in range(4) if not ins[q]]
            o = _even(ii + oo)
            i, j, kk, ll = (v[q] for q in o)
            q1 = [e(i, kk), e(i, ll), e(j, ll)]
            q2 = [e(i, kk), e(j, ll), e(j, kk)]
            if flip:
                q1 = [q1[0], q1[2], q1[1]]
                q2 = [q2[0], q2[2], q2[1]]
            tris += [q1, q2]
    return pts, np.asarray(tris, np.int64).reshape(-1, 3), ce
