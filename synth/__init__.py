"""Seeded synthetic inputs for the tetrahedron rasterizer.

This module builds the scene and camera arrays that both the HIP path and the
CPU oracle consume.  It holds none of the rendering method's arithmetic: no
projection, opacity, blending or gradient code lives here, only

* structured tetrahedral grids (Kuhn split of a cube grid; the paper renders a
  deformable tetrahedral grid, Sec. 3.1),
* per-vertex signed-distance fields of simple shapes plus seeded noise,
* per-vertex RGB,
* orbit cameras (OpenCV pinhole: +x right, +y down, +z forward).

Every array is produced once from ``numpy.random.default_rng(seed)`` and handed
to both sides as float32 / int32 arrays.

Camera packing (float32, one row of ``CAM_FIELDS`` per view)::

    [W, H, R00..R22 (row-major world->camera), t0, t1, t2,
     fx, fy, cx, cy, znear, bg_r, bg_g, bg_b]
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CAM_FIELDS = 22
ZNEAR = 0.01

# Axis permutations in lexicographic order; tet p of a cube walks the cube
# diagonal along axes perm[0], perm[1], perm[2].
_PERMS = np.array([(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)],
                  dtype=np.int64)


@dataclass
class Scene:
    verts: np.ndarray   # [V,3] float32
    tets: np.ndarray    # [K,4] int32
    sdf: np.ndarray     # [V]   float32
    colors: np.ndarray  # [V,3] float32
    s: float            # steepness of the SDF-to-opacity conversion
    name: str = ""
    res: int = 0

    @property
    def V(self) -> int:
        return int(self.verts.shape[0])

    @property
    def K(self) -> int:
        return int(self.tets.shape[0])


@dataclass
class Workload:
    name: str
    scenes: list
    cams: np.ndarray          # [n_views, CAM_FIELDS] float32
    view_scene: np.ndarray    # [n_views] int32: scene index of each view
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------
def kuhn_grid(R: int, lo: float = -1.0, hi: float = 1.0):
    """Cube grid of R^3 cells over [lo,hi]^3, each cell split into 6 tets.

    Vertex (x,y,z) has index x + (R+1)*(y + (R+1)*z).  Cell (x,y,z) has index
    q = x + R*(y + R*z); its tet p (0..5) has id 6q+p and vertices
    (v0, v0+e_a, v0+e_a+e_b, v0+(1,1,1)) for the p-th axis permutation (a,b,c)
    in lexicographic order.  The split is conforming across cells.
    """
    n = R + 1
    h = (hi - lo) / R
    ax = lo + h * np.arange(n, dtype=np.float64)
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    verts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)

    cz, cy, cx = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    base = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)  # [R^3,3] in cell order q
    stride = np.array([1, n, n * n], dtype=np.int64)
    v0 = base @ stride
    unit = np.eye(3, dtype=np.int64)
    tets = np.empty((R ** 3, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        s1 = unit[perm[0]] @ stride
        s2 = s1 + unit[perm[1]] @ stride
        tets[:, p, 0] = v0
        tets[:, p, 1] = v0 + s1
        tets[:, p, 2] = v0 + s2
        tets[:, p, 3] = v0 + stride.sum()
    return verts, tets.reshape(-1, 4).astype(np.int32)


# ----------------------------------------------------------------------------
# signed-distance fields (float64, cast by the caller)
# ----------------------------------------------------------------------------
def sdf_sphere(x: np.ndarray, r: float) -> np.ndarray:
    return np.linalg.norm(x, axis=1) - r


def sdf_torus_z(x: np.ndarray, R: float, r: float) -> np.ndarray:
    q = np.sqrt(x[:, 0] ** 2 + x[:, 1] ** 2) - R
    return np.sqrt(q * q + x[:, 2] ** 2) - r


def smooth_min(a: np.ndarray, b: np.ndarray, k: float) -> np.ndarray:
    """Polynomial smooth minimum: min(a,b) - h^2 k / 4, h = max(k-|a-b|,0)/k."""
    h = np.maximum(k - np.abs(a - b), 0.0) / k
    return np.minimum(a, b) - h * h * k * 0.25


def sdf_blob(x: np.ndarray, rng: np.random.Generator, bumps: int = 8) -> np.ndarray:
    """Sphere of radius 0.5 with Gaussian bumps on it (directions uniform on S^2)."""
    u = rng.normal(size=(bumps, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    amp = rng.uniform(0.05, 0.15, size=bumps)
    wid = rng.uniform(0.15, 0.35, size=bumps)
    r = np.linalg.norm(x, axis=1)
    xh = x / np.maximum(r, 1e-12)[:, None]
    rad = np.full(x.shape[0], 0.5)
    for k in range(bumps):
        d2 = np.sum((xh - u[k]) ** 2, axis=1)
        rad += amp[k] * np.exp(-d2 / (2.0 * wid[k] ** 2))
    return r - rad


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------
def orbit_camera(az: float, el: float, radius: float, fov_deg: float, W: int, H: int,
                 bg=(0.0, 0.0, 0.0), znear: float = ZNEAR) -> np.ndarray:
    """Pinhole camera on an orbit around the origin looking at it, up = +z.

    fx = fy = (W/2)/tan(fov/2), principal point at the image centre, pixel
    centres at (i+0.5, j+0.5).
    """
    C = radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    fwd = -C / np.linalg.norm(C)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    Rm = np.stack([right, down, fwd], axis=0)
    t = -Rm @ C
    f = (W / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    row = np.zeros(CAM_FIELDS, dtype=np.float64)
    row[0], row[1] = W, H
    row[2:11] = Rm.ravel()
    row[11:14] = t
    row[14], row[15], row[16], row[17] = f, f, W / 2.0, H / 2.0
    row[18] = znear
    row[19:22] = bg
    return row.astype(np.float32)


def random_orbit_cameras(rng: np.random.Generator, n: int, sizes, radius=2.5, fov_deg=50.0,
                         bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    """n cameras with azimuth ~ U[0,2pi), elevation ~ U[-30deg, 60deg]."""
    rows = []
    for i in range(n):
        az = rng.uniform(0.0, 2.0 * math.pi)
        el = math.radians(rng.uniform(-30.0, 60.0))
        W = H = int(sizes[i] if np.ndim(sizes) else sizes)
        rows.append(orbit_camera(az, el, radius, fov_deg, W, H, bg))
    return np.stack(rows, axis=0)


def cam_size(cam: np.ndarray):
    return int(cam[0]), int(cam[1])


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------
def band_prune(tets: np.ndarray, sdf: np.ndarray, band: float) -> np.ndarray:
    """Keep tets whose vertex SDF changes sign or comes within `band` of zero."""
    f = sdf[tets]
    keep = (f.min(axis=1) < 0) & (f.max(axis=1) > 0)
    keep |= np.abs(f).min(axis=1) < band
    return tets[keep]


def scene_sphere_noise(R: int, seed: int, s: float, radius=0.5, sigma=0.01) -> Scene:
    rng = np.random.default_rng(seed)
    verts, tets = kuhn_grid(R)
    sdf = sdf_sphere(verts, radius) + rng.normal(0.0, sigma, size=verts.shape[0])
    colors = rng.uniform(0.0, 1.0, size=(verts.shape[0], 3))
    return Scene(verts.astype(np.float32), tets, sdf.astype(np.float32),
                 colors.astype(np.float32), float(s), f"sphere{R}", R)


def scene_sphere_torus(R: int, seed: int, s: float, sigma=0.005) -> Scene:
    rng = np.random.default_rng(seed)
    verts, tets = kuhn_grid(R)
    f = smooth_min(sdf_sphere(verts, 0.4), sdf_torus_z(verts, 0.5, 0.15), 0.1)
    sdf = f + rng.normal(0.0, sigma, size=verts.shape[0])
    colors = rng.uniform(0.0, 1.0, size=(verts.shape[0], 3))
    return Scene(verts.astype(np.float32), tets, sdf.astype(np.float32),
                 colors.astype(np.float32), float(s), f"sphere_torus{R}", R)


def scene_blob(R: int, rng: np.random.Generator, s: float, band: float | None = 0.05) -> Scene:
    verts, tets = kuhn_grid(R)
    sdf = sdf_blob(verts, rng)
    colors = rng.uniform(0.0, 1.0, size=(verts.shape[0], 3))
    if band is not None:
        tets = band_prune(tets, sdf, band)
    return Scene(verts.astype(np.float32), tets, sdf.astype(np.float32),
                 colors.astype(np.float32), float(s), f"blob{R}", R)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------
def tiny(s: float = 20.0, bg=(0.0, 0.0, 0.0)) -> Workload:
    """8^3-cube grid (3072 tets, 729 verts), sphere r=0.5 + N(0,0.01), one 64^2 view."""
    sc = scene_sphere_noise(8, seed=0, s=s)
    cam = orbit_camera(0.7, 0.35, 2.5, 50.0, 64, 64, bg)[None]
    return Workload("tiny", [sc], cam, np.zeros(1, np.int32))


def training(s: float = 320.0, R: int = 64, size: int = 512, views: int = 4) -> Workload:
    """64^3-cube grid, smooth union of a sphere and a torus + N(0,0.005), 4 orbit views 512^2."""
    sc = scene_sphere_torus(R, seed=1, s=s)
    rng = np.random.default_rng(1001)
    cams = random_orbit_cameras(rng, views, size)
    return Workload("training", [sc], cams, np.zeros(views, np.int32))


def batched(s: float = 320.0, R: int = 128, size: int = 1024, views: int = 8) -> Workload:
    """128^3 blob grid pruned to the |f|<0.05 band, 8 views at 1024^2."""
    rng = np.random.default_rng(2)
    sc = scene_blob(R, rng, s)
    cams = random_orbit_cameras(rng, views, size)
    return Workload("batched", [sc], cams, np.zeros(views, np.int32))


def multiscene(s: float = 320.0, n_scenes: int = 32, res=(32, 48, 64, 96, 128),
               sizes=(256, 512, 768, 1024), max_views: int = 8, seed: int = 3) -> Workload:
    """Resident blob scenes of uneven tet counts, 1..max_views mixed-size views each."""
    rng = np.random.default_rng(seed)
    scenes, cams, owner = [], [], []
    for i in range(n_scenes):
        R = int(rng.choice(res))
        scenes.append(scene_blob(R, rng, s))
        nv = int(rng.integers(1, max_views + 1))
        sz = rng.choice(sizes, size=nv)
        cams.append(random_orbit_cameras(rng, nv, sz))
        owner += [i] * nv
    return Workload("multiscene", scenes, np.concatenate(cams, 0), np.array(owner, np.int32))


def serving_scenes(s: float = 320.0, n_scenes: int = 16, res=(32, 48, 64, 96, 128),
                   seed: int = 4) -> list:
    rng = np.random.default_rng(seed)
    return [scene_blob(int(rng.choice(res)), rng, s) for _ in range(n_scenes)]


def serving_requests(n: int, rate: float, n_scenes: int, sizes=(256, 512, 1024),
                     max_views: int = 4, seed: int = 5):
    """Open-loop Poisson arrivals: list of (arrival_s, scene, cams[nv, CAM_FIELDS])."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0 / rate)
        sc = int(rng.integers(0, n_scenes))
        nv = int(rng.integers(1, max_views + 1))
        sz = rng.choice(sizes, size=nv)
        out.append((t, sc, random_orbit_cameras(rng, nv, sz)))
    return out
