"""Independent float64 reference used only to pin the oracle.

It reaches the per-pixel quantities by a different route from the oracle:
instead of 2D barycentrics on projected faces plus perspective correction
(App. A.1-A.2), it intersects the pixel's 3D camera ray with the tet's face
planes, tests the hit point with 3D barycentrics, and evaluates the linear SDF
at the hit points directly.  Opacity uses the literal Eq. 1 with Python's
exact-enough math on logistic functions evaluated as ratios.
"""
from __future__ import annotations

import math

import numpy as np

FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))


def cam_parts(cam):
    cam = np.asarray(cam, np.float64)
    R = cam[2:11].reshape(3, 3)
    t = cam[11:14]
    fx, fy, cx, cy = cam[14:18]
    return R, t, fx, fy, cx, cy


def ray_dir(cam, qx, qy):
    _, _, fx, fy, cx, cy = cam_parts(cam)
    return np.array([(qx - cx) / fx, (qy - cy) / fy, 1.0])


def ray_tet(Xc, f, d):
    """Ray o + t d (o = 0) against a tet with camera-space vertices Xc [4,3].

    Returns None or (t_entry, t_exit, f_entry, f_exit).  A face is hit if the
    ray meets its plane at a point whose 3D barycentrics are all >= 0.
    """
    hits = []
    for (a, b, c) in FACES:
        A, B, C = Xc[a], Xc[b], Xc[c]
        n = np.cross(B - A, C - A)
        den = n @ d
        if den == 0.0:
            continue
        t = (n @ A) / den
        P = t * d
        nn = n @ n
        la = np.cross(B - P, C - P) @ n / nn
        lb = np.cross(C - P, A - P) @ n / nn
        lc = np.cross(A - P, B - P) @ n / nn
        if la >= 0 and lb >= 0 and lc >= 0:
            hits.append((t, la * f[a] + lb * f[b] + lc * f[c]))
    if len(hits) < 2:
        return None
    ent = min(hits, key=lambda h: h[0])
    ext = max(hits, key=lambda h: h[0])
    return ent[0], ext[0], ent[1], ext[1]


def logistic(x, s):
    # 1 / (1 + e^{-s x}) without overflow
    z = -s * x
    if z > 700:
        return math.exp(-z)
    return 1.0 / (1.0 + math.exp(z))


def alpha_literal(fp, fn, s):
    """Eq. 1 exactly as printed (float64); may be nan where it underflows."""
    pp, pn = logistic(fp, s), logistic(fn, s)
    if pp == 0.0:
        return float("nan")
    return max((pp - pn) / pp, 0.0)


def render_ray_route(verts, tets, sdf, colors, cam, s, alpha_min, alpha_clamp, t_min, keep):
    """Whole-image forward by the 3D ray route.  Returns out [8,H,W] and the
    set of pixels whose blend order involves a near-tie of tet depths."""
    R, t, fx, fy, cx, cy = cam_parts(cam)
    W, H = int(cam[0]), int(cam[1])
    bg = np.asarray(cam[19:22], np.float64)
    V = np.asarray(verts, np.float64)
    F = np.asarray(sdf, np.float64)
    Cc = np.asarray(colors, np.float64)
    Xc_all = V @ R.T + t
    per_pix = {}
    for k in np.nonzero(keep)[0]:
        tv = tets[k]
        Xc = Xc_all[tv]
        if np.any(Xc[:, 2] < cam[18]):
            continue
        px = fx * Xc[:, 0] / Xc[:, 2] + cx
        py = fy * Xc[:, 1] / Xc[:, 2] + cy
        i0 = max(0, math.ceil(px.min() - 0.5))
        i1 = min(W - 1, math.floor(px.max() - 0.5))
        j0 = max(0, math.ceil(py.min() - 0.5))
        j1 = min(H - 1, math.floor(py.max() - 0.5))
        f = F[tv]
        # normal from the 3x3 edge system (a different route from App. A.3)
        E = (V[tv[1:]] - V[tv[0]])
        g = np.linalg.solve(E, f[1:] - f[0])
        gn = np.linalg.norm(g)
        nrm = g / gn if gn > 0 else np.zeros(3)
        col = Cc[tv].mean(axis=0)
        zt = Xc[:, 2].mean()
        for j in range(j0, j1 + 1):
            for i in range(i0, i1 + 1):
                d = ray_dir(cam, i + 0.5, j + 0.5)
                h = ray_tet(Xc, f, d)
                if h is None:
                    continue
                fp, fn = h[2], h[3]
                a = alpha_literal(fp, fn, s)
                per_pix.setdefault((i, j), []).append((zt, int(k), a, col, nrm))
    out = np.zeros((8, H, W))
    out[0:3] = bg[:, None, None]
    ties = set()
    for (i, j), lst in per_pix.items():
        lst.sort(key=lambda e: (e[0], e[1]))
        for q in range(1, len(lst)):
            if abs(lst[q][0] - lst[q - 1][0]) < 1e-6 * abs(lst[q][0]):
                ties.add((i, j))
        T = 1.0
        acc = np.zeros(8)
        for zt, k, a, col, nrm in lst:
            if a < alpha_min:
                continue
            a = min(a, alpha_clamp)
            Tn = T * (1 - a)
            if Tn < t_min:
                break
            w = T * a
            acc[0:3] += w * col
            acc[3] += w
            acc[4] += w * zt
            acc[5:8] += w * nrm
            T = Tn
            if T == 0.0:
                break
        acc[0:3] += T * bg
        out[:, j, i] = acc
    return out, ties
