"""Pins of the Marching Tetrahedra oracle against geometry fixed outside it:
a plane cut through the cube grid (points on the plane, exact area, normals
along the SDF gradient), a sphere (closed, consistently oriented, Euler
characteristic 2, inscribed, enclosed volume just under 4/3 pi r^3), and every inside/outside
pattern of a single tet in both orientations (triangle count, zero of the
interpolant at each point, outward normals by a geometric test)."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import marching_tets as MT


def _normals(pts, tris):
    p = pts[tris]
    return np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])


@pytest.mark.parametrize("tilt", [0.0, 0.3])
def test_plane_cut(tilt):
    verts, tets = synth.kuhn_grid(4)
    n = np.array([tilt, 0.0, 1.0])
    c = 0.1234
    sdf = verts @ n - c
    pts, tris, _ = MT.extract(verts, tets, sdf)
    assert np.abs(pts @ n - c).max() < 1e-12
    nr = _normals(pts, tris)
    area = 0.5 * np.linalg.norm(nr, axis=1).sum()
    assert area == pytest.approx(4.0 * math.sqrt(1.0 + tilt * tilt), rel=1e-12)
    assert (nr @ n > 0).all()


def test_sphere_is_closed_oriented_and_encloses_the_ball():
    verts, tets = synth.kuhn_grid(12)
    r = 0.61
    sdf = np.linalg.norm(verts, axis=1) - r
    pts, tris, _ = MT.extract(verts, tets, sdf)
    directed = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], 0)
    assert len({tuple(e) for e in directed}) == len(directed)          # each directed edge once
    und = {tuple(sorted(e)) for e in directed}
    assert all((b, a) in {tuple(e) for e in directed} for a, b in directed)   # and its reverse too
    assert len(pts) - len(und) + len(tris) == 2
    p = pts[tris]
    vol = np.einsum("ij,ij->i", p[:, 0], np.cross(p[:, 1], p[:, 2])).sum() / 6.0
    # the interpolant of the convex |x| lies above it along an edge, so every
    # point is inside the sphere and the mesh is inscribed: volume below the
    # ball's, by an O(h^2) amount
    assert np.linalg.norm(pts, axis=1).max() <= r + 1e-12
    ball = 4.0 / 3.0 * math.pi * r ** 3
    assert 0.94 * ball < vol < ball


@pytest.mark.parametrize("neg", [False, True])
def test_every_sign_pattern_of_one_tet(neg):
    x = np.array([[0.0, 0, 0], [1, 0.1, 0], [0.2, 1, 0], [0.1, 0.3, 1]])
    if neg:
        x = x[[0, 2, 1, 3]]                                             # negatively oriented
    tets = np.array([[0, 1, 2, 3]])
    rng = np.random.default_rng(0)
    for bits in itertools.product([0, 1], repeat=4):
        f = np.where(np.array(bits) == 1, -rng.uniform(0.2, 1.0, 4), rng.uniform(0.2, 1.0, 4))
        pts, tris, ce = MT.extract(x, tets, f)
        c = sum(bits)
        assert len(tris) == {0: 0, 1: 1, 2: 2, 3: 1, 4: 0}[c]
        assert len(pts) == {0: 0, 1: 3, 2: 4, 3: 3, 4: 0}[c]
        # the interpolant of f along each crossed edge vanishes at its point
        for q, (a, b) in zip(pts, ce):
            t = np.dot(q - x[a], x[b] - x[a]) / np.dot(x[b] - x[a], x[b] - x[a])
            assert abs((1 - t) * f[a] + t * f[b]) < 1e-12
        if c in (1, 2, 3):
            ins = np.array(bits) == 1
            out_dir = x[~ins].mean(0) - x[ins].mean(0)
            assert (_normals(pts, tris) @ out_dir > 0).all()
