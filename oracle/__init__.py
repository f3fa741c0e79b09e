"""ctypes front end of the plain CPU oracle (``tetsplat_oracle.cpp``).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
package never imports it and shares no code with it.

Functions that have no independent pin are listed in the module docstring of
the C++ file; every function here is pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tetsplat_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# (tile_w, tile_h, alpha_min, alpha_clamp, t_min, prefilter_tf)
DEFAULT = dict(tile_w=16, tile_h=16, alpha_min=1.0 / 255.0, alpha_clamp=0.99, t_min=1e-4,
               prefilter_tf=1.0 / 255.0, window=0)
# thresholds off: the rendered function is piecewise smooth
EXACT = dict(DEFAULT, alpha_min=0.0, alpha_clamp=1.0, t_min=0.0)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-mavx2", "-mfma",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_render.argtypes = [C.c_int, P, P, P, P, C.c_int, C.c_int, P, C.c_int, P, P, C.c_long, P, P, P]
        L.oracle_render_dual.argtypes = [P, P, P, P, C.c_int, C.c_int, P, P, P, P, C.c_int, P, P, C.c_long, P, P]
        L.oracle_backward.argtypes = [C.c_int, P, P, P, P, C.c_int, C.c_int, P, C.c_int, P, P, C.c_long, P, P, P, P]
        L.oracle_render_errbound.argtypes = [P, P, P, P, C.c_int, C.c_int, P, C.c_int, P, P, C.c_long, P, P]
        L.oracle_alpha_errbound.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.oracle_alpha_errbound.restype = C.c_double
        L.oracle_backward_budget.argtypes = [P, P, P, P, C.c_int, C.c_int, P, C.c_int, P, P, C.c_long, P,
                                             P, P, P]
        L.oracle_prefilter.argtypes = [C.c_int, P, P, P, P, C.c_int, C.c_int, P, P, P, P, P, P]
        L.oracle_binning.argtypes = [P, P, P, C.c_int, C.c_int, P, C.c_int, P, C.c_long, P, P, P, P, P]
        L.oracle_binning.restype = C.c_long
        L.oracle_pixel_trace.argtypes = [C.c_int, P, P, P, P, C.c_int, C.c_int, P, C.c_int, P, C.c_int,
                                         C.c_int, C.c_int, C.c_int, P, P, P, P, P, P, P]
        L.oracle_pixel_decisions.argtypes = [P, P, P, P, C.c_int, C.c_int, P, C.c_int, P, C.c_int, C.c_int,
                                             C.c_int, C.c_int, P, P, P, P]
        L.oracle_tet_pixel.argtypes = [P, P, P, P, C.c_double, C.c_double, C.c_double, P]
        L.oracle_alpha.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_alpha.restype = C.c_double
        L.oracle_alpha_f32.argtypes = [C.c_float, C.c_float, C.c_float]
        L.oracle_alpha_f32.restype = C.c_float
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the count in effect."""
    return int(lib().oracle_set_threads(int(n)))


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params_array(s: float, **kw) -> np.ndarray:
    d = dict(DEFAULT)
    d.update(kw)
    return np.array([d["tile_w"], d["tile_h"], d["alpha_min"], d["alpha_clamp"], d["t_min"],
                     d["prefilter_tf"], s, d["window"]], dtype=np.float32)


class Geometry:
    """Scene arrays held in float64 for the oracle (inputs are float32 values)."""

    def __init__(self, verts, tets, sdf, colors):
        self.verts = _f64(verts)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.sdf = _f64(sdf)
        self.colors = _f64(colors)
        self.V = int(self.verts.shape[0])
        self.K = int(self.tets.shape[0])

    @classmethod
    def of(cls, scene):
        return cls(scene.verts, scene.tets, scene.sdf, scene.colors)


def all_pixels(cams: np.ndarray, views=None) -> np.ndarray:
    rows = []
    for v in (range(cams.shape[0]) if views is None else views):
        W, H = int(cams[v, 0]), int(cams[v, 1])
        jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        rows.append(np.stack([np.full(W * H, v), ii.ravel(), jj.ravel()], axis=1))
    return np.ascontiguousarray(np.concatenate(rows, 0), dtype=np.int32)


def render(g: Geometry, cams, params, pix=None, prec: int = 64, want_state: bool = False):
    """Outputs [npix, 8] (R,G,B,O,D,Nx,Ny,Nz) for the listed (view, i, j) pixels."""
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    if pix is None:
        pix = all_pixels(cams)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    n = pix.shape[0]
    out = np.zeros((n, 8), np.float64)
    nb = np.zeros(n, np.int32)
    tf = np.zeros(n, np.float64)
    rc = lib().oracle_render(prec, _p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(cams),
                             cams.shape[0], _p(params), _p(pix), n, _p(out), _p(nb), _p(tf))
    assert rc == 0
    return (out, nb, tf) if want_state else out


def render_images(g: Geometry, cams, params, prec: int = 64):
    """Full images as a list of [8,H,W] arrays, one per view."""
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    pix = all_pixels(cams)
    out = render(g, cams, params, pix, prec)
    imgs, o = [], 0
    for v in range(cams.shape[0]):
        W, H = int(cams[v, 0]), int(cams[v, 1])
        imgs.append(out[o:o + W * H].reshape(H, W, 8).transpose(2, 0, 1).copy())
        o += W * H
    return imgs


def render_dual(g: Geometry, cams, params, pix, tverts=None, tsdf=None, tcolors=None):
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    n = pix.shape[0]
    out = np.zeros((n, 8), np.float64)
    tout = np.zeros((n, 8), np.float64)
    tv = None if tverts is None else _f64(tverts)
    ts = None if tsdf is None else _f64(tsdf)
    tc = None if tcolors is None else _f64(tcolors)
    lib().oracle_render_dual(_p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(tv), _p(ts), _p(tc),
                             _p(cams), cams.shape[0], _p(params), _p(pix), n, _p(out), _p(tout))
    return out, tout


def backward(g: Geometry, cams, params, pix, dout, prec: int = 64):
    """(dverts [V,3], dsdf [V], dcolors [V,3]) for upstream dL/dout [npix,8]."""
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    dout = _f64(dout)
    dv = np.zeros((g.V, 3), np.float64)
    ds = np.zeros(g.V, np.float64)
    dc = np.zeros((g.V, 3), np.float64)
    rc = lib().oracle_backward(prec, _p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(cams),
                               cams.shape[0], _p(params), _p(pix), pix.shape[0], _p(dout), _p(dv), _p(ds), _p(dc))
    assert rc == 0
    return dv, ds, dc


def render_error_bound(g: Geometry, cams, params, pix):
    """(out [npix, 8] float64, bound [npix, 8]): the running error bound of a
    float32 evaluation of ``render`` (first order, per channel)."""
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    n = pix.shape[0]
    out = np.zeros((n, 8), np.float64)
    bnd = np.zeros((n, 8), np.float64)
    lib().oracle_render_errbound(_p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(cams),
                                 cams.shape[0], _p(params), _p(pix), n, _p(out), _p(bnd))
    return out, bnd


def alpha_error_bound(fprev, fnext, s):
    """(alpha, bound): Eq. 1 in float64 and the running error bound of its float32 evaluation."""
    b = np.zeros(1, np.float64)
    a = lib().oracle_alpha_errbound(float(fprev), float(fnext), float(s), _p(b))
    return float(a), float(b[0])


def backward_budget(g: Geometry, cams, params, pix, dout):
    """Error budget of a float32 evaluation of ``backward`` (float64 arrays,
    each split as (dverts [V,3], dsdf [V], dcolors [V,3])):

    A -- sum over (view, tet) of |J| times the summed per-pixel |g|: any order
         and grouping of the float32 sums moves an element by at most
         gamma_{n-1} A (Higham, Sec. 4.2, carried through the linear chain);
    E -- sum over (view, tet) of |J| times the summed running error bounds of
         the per-pixel terms (a term only one precision blends: in full);
    N -- number of terms reaching the element.
    """
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    dout = _f64(dout)
    A, E, N = (np.zeros((g.V, 7), np.float64) for _ in range(3))
    rc = lib().oracle_backward_budget(_p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(cams),
                                      cams.shape[0], _p(params), _p(pix), pix.shape[0], _p(dout), _p(A), _p(E),
                                      _p(N))
    assert rc == 0

    def split(x):
        return x[:, 0:3].copy(), x[:, 3].copy(), x[:, 4:7].copy()
    return dict(A=split(A), E=split(E), N=split(N))


def prefilter(g: Geometry, params, prec: int = 64):
    """keep [K] bool, alpha_max (float32 decision value) [K], normal [K,3], color [K,3], grad [K,3]."""
    K = g.K
    keep = np.zeros(K, np.uint8)
    amax = np.zeros(K, np.float32)
    nrm = np.zeros((K, 3), np.float64)
    col = np.zeros((K, 3), np.float64)
    grd = np.zeros((K, 3), np.float64)
    rc = lib().oracle_prefilter(prec, _p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, K, _p(params),
                                _p(keep), _p(amax), _p(nrm), _p(col), _p(grd))
    assert rc == 0
    return keep.astype(bool), amax, nrm, col, grd


def binning(g: Geometry, cams, params, want_rect: bool = False):
    """Reference tiling: dict(tile, zbits, tet, ranges[, rect]) in sorted order."""
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    L = lib()
    nv = cams.shape[0]
    tw, th = int(params[0]), int(params[1])
    ntiles = sum(((int(c[0]) + tw - 1) // tw) * ((int(c[1]) + th - 1) // th) for c in cams)
    E = L.oracle_binning(_p(g.verts), _p(g.tets), _p(g.sdf), g.V, g.K, _p(cams), nv, _p(params), 0,
                         None, None, None, None, None)
    tile = np.zeros(E, np.int32)
    zb = np.zeros(E, np.uint32)
    tet = np.zeros(E, np.int32)
    ranges = np.zeros((ntiles, 2), np.int32)
    rect = np.zeros((nv, g.K, 4), np.int32) if want_rect else None
    E2 = L.oracle_binning(_p(g.verts), _p(g.tets), _p(g.sdf), g.V, g.K, _p(cams), nv, _p(params), E,
                          _p(tile), _p(zb), _p(tet), _p(ranges), _p(rect))
    assert E2 == E
    d = dict(tile=tile, zbits=zb, tet=tet, ranges=ranges, E=E, ntiles=ntiles)
    if want_rect:
        d["rect"] = rect
    return d


def pixel_trace(g: Geometry, cams, params, view, i, j, prec: int = 64, cap: int = 4096):
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    tid = np.zeros(cap, np.int32)
    a, T, ar, fp, fn, zi = (np.zeros(cap, np.float64) for _ in range(6))
    n = lib().oracle_pixel_trace(prec, _p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(cams),
                                 cams.shape[0], _p(params), view, i, j, cap, _p(tid), _p(a), _p(T), _p(ar),
                                 _p(fp), _p(fn), _p(zi))
    n = min(n, cap)
    return dict(tet=tid[:n], alpha=a[:n], T=T[:n], alpha_raw=ar[:n], fprev=fp[:n], fnext=fn[:n], zin=zi[:n])


def pixel_decisions(g: Geometry, cams, params, view, i, j, cap: int = 8192):
    """Threshold decisions of one pixel's walk: dict(kind, value, bound,
    threshold) with kind 0 = alpha vs alpha_min, 1 = alpha vs alpha_clamp,
    2 = T (1 - alpha) vs t_min; value in float64 and bound the running error
    bound of a float32 evaluation of it."""
    cams = np.ascontiguousarray(cams, dtype=np.float32)
    kind = np.zeros(cap, np.int32)
    val, bnd, thr = (np.zeros(cap, np.float64) for _ in range(3))
    n = lib().oracle_pixel_decisions(_p(g.verts), _p(g.tets), _p(g.sdf), _p(g.colors), g.V, g.K, _p(cams),
                                     cams.shape[0], _p(params), int(view), int(i), int(j), cap, _p(kind), _p(val),
                                     _p(bnd), _p(thr))
    n = min(n, cap)
    return dict(kind=kind[:n], value=val[:n], bound=bnd[:n], threshold=thr[:n])


def tet_pixel(px, py, Z, f, qx, qy, s):
    """(hit, f_prev, f_next, z_entry, z_exit, alpha) of one projected tet at one point."""
    out = np.zeros(6, np.float64)
    a = [_f64(x) for x in (px, py, Z, f)]
    lib().oracle_tet_pixel(_p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), float(qx), float(qy), float(s), _p(out))
    return out


def alpha(fprev, fnext, s) -> float:
    return float(lib().oracle_alpha(float(fprev), float(fnext), float(s)))


def alpha_f32(fprev, fnext, s) -> float:
    return float(lib().oracle_alpha_f32(float(fprev), float(fnext), float(s)))
