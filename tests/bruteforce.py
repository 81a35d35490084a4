"""Independent brute-force references for the renderer (Section 3.3.1):

* ``exact_coverage``: exact rational point-in-triangle of every pixel centre
  against snapped triangles, with the top/left tie rule expressed through
  barycentric gradients (an on-edge centre belongs to the triangle whose
  interior lies on its +x side, or, for a horizontal edge, below it);
* ``exact_project``: exact rational projection and round-half-even snap;
* ``raycast64``: a binary64 ray cast (Moller-Trumbore) of every pixel centre
  against the unclipped 3-D triangles, with a stability flag for pixels whose
  nearest hit changes under a 1/100-pixel jitter.

No code is shared with the oracle or the HIP library.
"""
from fractions import Fraction

import numpy as np


def exact_project(cam, X):
    """Snapped (X, Y) of a world point with an exactly representable camera."""
    fx, fy, cx, cy = (Fraction(float(v)) for v in cam[:4])
    R = [Fraction(float(v)) for v in cam[4:13]]
    t = [Fraction(float(v)) for v in cam[13:16]]
    P = [Fraction(float(v)) for v in X]
    xc = R[0] * P[0] + R[1] * P[1] + R[2] * P[2] + t[0]
    yc = R[3] * P[0] + R[4] * P[1] + R[5] * P[2] + t[1]
    zc = R[6] * P[0] + R[7] * P[1] + R[8] * P[2] + t[2]
    px = fx * xc / zc + cx
    py = fy * yc / zc + cy
    return round(px * 256), round(py * 256), zc   # Python rounds Fractions half to even


def _bary(tri, P):
    (x0, y0), (x1, y1), (x2, y2) = tri
    den = Fraction((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0))
    px, py = P
    l1 = Fraction((px - x0) * (y2 - y0) - (x2 - x0) * (py - y0)) / den
    l2 = Fraction((x1 - x0) * (py - y0) - (px - x0) * (y1 - y0)) / den
    return [1 - l1 - l2, l1, l2]


def _grad(tri, i):
    """Gradient of barycentric coordinate i (points into the triangle)."""
    (x0, y0), (x1, y1), (x2, y2) = tri
    den = Fraction((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0))
    g1 = (Fraction(y2 - y0) / den, Fraction(-(x2 - x0)) / den)
    g2 = (Fraction(-(y1 - y0)) / den, Fraction(x1 - x0) / den)
    if i == 1:
        return g1
    if i == 2:
        return g2
    return (-g1[0] - g2[0], -g1[1] - g2[1])


def covers(tri, P):
    """Exact coverage of pixel centre P (sub-pixel integer coordinates)."""
    (x0, y0), (x1, y1), (x2, y2) = tri
    if (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0) == 0:
        return False
    lam = _bary(tri, P)
    for i in range(3):
        if lam[i] < 0:
            return False
        if lam[i] == 0:
            gx, gy = _grad(tri, i)
            if not (gx > 0 or (gx == 0 and gy > 0)):
                return False
    return True


def exact_coverage(snapped, H, W):
    """snapped: list of (triangle id, [(X,Y)]*3).  Returns count [H,W] and
    the list of covering ids per pixel."""
    cnt = np.zeros((H, W), np.int32)
    who = [[[] for _ in range(W)] for _ in range(H)]
    for tid, tri in snapped:
        xs = [p[0] for p in tri]
        ys = [p[1] for p in tri]
        x0 = max(0, min(xs) // 256 - 1)
        x1 = min(W - 1, max(xs) // 256 + 1)
        y0 = max(0, min(ys) // 256 - 1)
        y1 = min(H - 1, max(ys) // 256 + 1)
        for y in range(y0, y1 + 1):
            for x in range(x0, x1 + 1):
                if covers(tri, (256 * x + 128, 256 * y + 128)):
                    cnt[y, x] += 1
                    who[y][x].append(tid)
    return cnt, who


def exact_plane_depth(cam, tri3d, x, y):
    """Exact camera depth of the plane of a 3-D triangle along the ray of
    pixel (x, y), for an exactly representable camera."""
    fx, fy, cx, cy = (Fraction(float(v)) for v in cam[:4])
    R = [Fraction(float(v)) for v in cam[4:13]]
    t = [Fraction(float(v)) for v in cam[13:16]]

    def tc(P):
        P = [Fraction(float(v)) for v in P]
        return [R[3 * r] * P[0] + R[3 * r + 1] * P[1] + R[3 * r + 2] * P[2] + t[r] for r in range(3)]

    A, B, Cc = (tc(p) for p in tri3d)
    e1 = [B[i] - A[i] for i in range(3)]
    e2 = [Cc[i] - A[i] for i in range(3)]
    n = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
    r = [(Fraction(x) + Fraction(1, 2) - cx) / fx, (Fraction(y) + Fraction(1, 2) - cy) / fy, Fraction(1)]
    den = sum(n[i] * r[i] for i in range(3))
    if den == 0:
        return None
    return sum(n[i] * A[i] for i in range(3)) / den


# --------------------------------------------------------------------------- binary64 ray cast

def _rays(cam, H, W, jx=0.0, jy=0.0):
    fx, fy, cx, cy = (float(v) for v in cam[:4])
    xs = (np.arange(W) + 0.5 + jx - cx) / fx
    ys = (np.arange(H) + 0.5 + jy - cy) / fy
    d = np.stack(np.broadcast_arrays(xs[None, :], ys[:, None], np.ones((H, W))), -1)
    return d  # camera space, z = 1


def _cam_tris(cam, V, Fc):
    R = np.asarray(cam[4:13], np.float64).reshape(3, 3)
    t = np.asarray(cam[13:16], np.float64)
    Vc = np.asarray(V, np.float64) @ R.T + t
    return Vc[np.asarray(Fc)]


def _nearest(tris, d, z_near):
    """Nearest hit (triangle index, depth) per ray; -1 where none."""
    H, W, _ = d.shape
    best_t = np.full((H, W), np.inf)
    best_i = np.full((H, W), -1, np.int64)
    for i, (A, B, C) in enumerate(tris):
        e1, e2 = B - A, C - A
        p = np.cross(d, e2)
        det = p @ e1
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / det
            s = -A
            u = (p @ s) * inv
            q = np.cross(s, e1)
            v = (d @ q) * inv
            z = (q @ e2) * inv  # ray parameter = camera depth since d_z = 1
        ok = (det != 0) & (u >= 0) & (v >= 0) & (u + v <= 1) & (z >= z_near) & (z < best_t)
        best_t = np.where(ok, z, best_t)
        best_i = np.where(ok, i, best_i)
    return best_i, best_t


def raycast64(cam, V, F, H, W, z_near=0.05, jitter=0.01):
    """Nearest triangle and depth per pixel in binary64, plus a mask of
    pixels whose answer is stable under +-jitter pixel shifts."""
    tris = _cam_tris(cam, V, F)
    i0, t0 = _nearest(tris, _rays(cam, H, W), z_near)
    stable = np.ones((H, W), bool)
    for jx, jy in ((jitter, 0), (-jitter, 0), (0, jitter), (0, -jitter)):
        i1, _ = _nearest(tris, _rays(cam, H, W, jx, jy), z_near)
        stable &= i1 == i0
    # depth ties / near-plane grazing: also unstable if the second-nearest is within 1e-6 relative
    return i0, t0, stable
