"""Pins of the oracle renderer (Section 3.3.1, eq. projected-pixels,
eq. idtexel) against independent brute force: exact rational coverage on
two-triangle scenes, a binary64 ray cast, watertightness.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from tests import bruteforce as bf

W, H = 64, 48
CAM_EXACT = np.array([64, 64, 32, 24, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def _world(Xs, Ys, z):
    """World point whose projection by CAM_EXACT is exactly (Xs, Ys)/256 px."""
    x = (Xs / 256.0 - 32.0) * z / 64.0
    y = (Ys / 256.0 - 24.0) * z / 64.0
    p = np.array([x, y, z], np.float32)
    assert float(p[0]) == x and float(p[1]) == y
    return p


def _mesh(tris3d, s=1, scheme=oracle.SPLIT):
    V = np.concatenate(tris3d).astype(np.float32)
    F = np.arange(V.shape[0], dtype=np.int32).reshape(-1, 3)
    return oracle.Mesh(V, F, s=s, scheme=scheme), V, F


def _exact_winner(mesh, V, F, cam):
    snapped = []
    depth = {}
    for t in range(F.shape[0]):
        pts = [bf.exact_project(cam, V[F[t, m]]) for m in range(3)]
        snapped.append((t, [(p[0], p[1]) for p in pts]))
        # the oracle's own snapped vertices must equal the exact ones
        fan = mesh.snapped_fan(t, cam)
        assert fan.shape[0] == 1
        assert sorted(map(tuple, fan[0].tolist())) == sorted((p[0], p[1]) for p in pts)
    cnt, who = bf.exact_coverage(snapped, H, W)
    ref = np.full((H, W), -1, np.int32)
    for y in range(H):
        for x in range(W):
            if who[y][x]:
                cands = [(bf.exact_plane_depth(cam, [V[F[t, m]] for m in range(3)], x, y), t) for t in who[y][x]]
                cands = [c for c in cands if c[0] is not None and c[0] > 0]
                if cands:
                    ref[y, x] = min(cands)[1]
    return ref, cnt


def test_exact_random_frontoparallel_scenes():
    """Random overlapping triangles on planes z in {1,2,4}, vertices with 10
    sub-pixel bits (so the snap rounds, including exact halves): triangle ids
    equal the exact rational reference on every pixel."""
    rng = np.random.default_rng(11)
    for scene in range(6):
        tris = []
        for t in range(10):
            z = float(rng.choice([1.0, 2.0, 4.0]))
            pts = []
            for m in range(3):
                X = int(rng.integers(-40 * 1024, (W + 40) * 1024)) / 4.0
                Y = int(rng.integers(-40 * 1024, (H + 40) * 1024)) / 4.0
                pts.append(_world(X, Y, z))
            tris.append(np.stack(pts))
        mesh, V, F = _mesh(tris)
        tri, l, z = mesh.raster(CAM_EXACT, H, W)
        ref, _ = _exact_winner(mesh, V, F, CAM_EXACT)
        assert np.array_equal(tri, ref), f"scene {scene}: {np.argwhere(tri != ref)[:5]}"


def _grid_tris(nx, ny, x0, y0, step, z, perturb=None, rng=None):
    pts = {}
    for j in range(ny + 1):
        for i in range(nx + 1):
            X, Y = x0 + i * step, y0 + j * step
            pts[(i, j)] = (X, Y)
    tris = []
    for j in range(ny):
        for i in range(nx):
            a, b, c, d = pts[(i, j)], pts[(i + 1, j)], pts[(i + 1, j + 1)], pts[(i, j + 1)]
            tris.append(np.stack([_world(*a, z), _world(*b, z), _world(*c, z)]))
            tris.append(np.stack([_world(*a, z), _world(*c, z), _world(*d, z)]))
    return tris


def test_shared_edges_through_pixel_centres_claimed_once():
    # grid vertices on pixel centres: every shared edge (horizontal, vertical,
    # diagonal) passes through pixel centres
    tris = _grid_tris(6, 4, 256 * 4 + 128, 256 * 5 + 128, 256 * 7, 2.0)
    mesh, V, F = _mesh(tris)
    cnt = mesh.coverage_count(CAM_EXACT, H, W)
    ref_tri, ref_cnt = _exact_winner(mesh, V, F, CAM_EXACT)
    assert np.array_equal(cnt, ref_cnt)
    assert cnt.max() == 1
    # the interior of the grid (pixel centres strictly inside or on the
    # top/left outer border) is covered exactly once
    inner = cnt[5:5 + 28, 4:4 + 42]
    assert (inner == 1).all()
    tri, _, _ = mesh.raster(CAM_EXACT, H, W)
    assert np.array_equal(tri, ref_tri)


def test_fan_around_vertex_on_pixel_centre():
    c = (256 * 20 + 128, 256 * 20 + 128)
    ring = []
    for k in range(7):
        a = 2 * math.pi * k / 7
        ring.append((c[0] + int(round(2000 * math.cos(a))), c[1] + int(round(2000 * math.sin(a)))))
    tris = [np.stack([_world(*c, 2.0), _world(*ring[k], 2.0), _world(*ring[(k + 1) % 7], 2.0)]) for k in range(7)]
    mesh, V, F = _mesh(tris)
    cnt = mesh.coverage_count(CAM_EXACT, H, W)
    assert cnt[20, 20] == 1
    assert cnt.max() == 1
    _, ref_cnt = _exact_winner(mesh, V, F, CAM_EXACT)
    assert np.array_equal(cnt, ref_cnt)


def test_occlusion_coplanar_tie_degenerate_sliver_offscreen():
    big = [(256 * 2, 256 * 2), (256 * 60, 256 * 3), (256 * 10, 256 * 45)]
    tris = [
        np.stack([_world(*p, 4.0) for p in big]),                    # 0: far
        np.stack([_world(*p, 2.0) for p in big[::-1]]),              # 1: near, same footprint
        np.stack([_world(*p, 2.0) for p in big]),                    # 2: coplanar with 1 -> 1 wins (lower id)
        np.stack([_world(256 * 5, 256 * 5, 1.0), _world(256 * 30, 256 * 30, 1.0),
                  _world(256 * 55, 256 * 55, 1.0)]),                 # 3: degenerate (collinear)
        np.stack([_world(256 * 3, 256 * 40, 1.0), _world(256 * 60 + 77, 256 * 40 + 100, 1.0),
                  _world(256 * 60, 256 * 40 + 300, 1.0)]),           # 4: sliver, nearest
        np.stack([_world(-256 * 30, 256 * 10, 1.0), _world(256 * 10, 256 * 12, 1.0),
                  _world(-256 * 5, 256 * 70, 1.0)]),                 # 5: partly off-screen
    ]
    mesh, V, F = _mesh(tris)
    tri, _, z = mesh.raster(CAM_EXACT, H, W)
    ref, _ = _exact_winner(mesh, V, F, CAM_EXACT)
    assert np.array_equal(tri, ref)
    assert not (tri == 0).any() and not (tri == 2).any() and not (tri == 3).any()
    assert (tri == 1).sum() > 100 and (tri == 4).any() and (tri == 5).any()
    assert np.all(z[tri == 1] == 2.0)


def _random_cam(rng, W, H, pos=None, target=None):
    from paper_2111_11103_amd.scenes import camera_matrix
    pos = rng.uniform(-1, 1, 3) if pos is None else pos
    target = rng.uniform(-1, 1, 3) + np.array([0, 0, 0.0]) if target is None else target
    return camera_matrix(pos, target, W, H, up=(0.0, 0.0, 1.0))


def test_raycast64_random_tilted_scenes():
    """Nearest triangle per pixel equals a binary64 ray cast wherever the
    ray-cast answer is stable under 1/100-pixel jitter; depth within 1e-5
    relative; texel cell equals the binary64 uv's cell away from cell borders."""
    rng = np.random.default_rng(3)
    Wr, Hr = 80, 60
    n_checked = 0
    for scene in range(5):
        V = rng.uniform(-2, 2, (24, 3)).astype(np.float32)
        F = np.arange(24, dtype=np.int32).reshape(8, 3)
        s = int(rng.integers(1, 5))
        scheme = int(rng.integers(0, 2))
        mesh = oracle.Mesh(V, F, s=s, scheme=scheme)
        cam = _random_cam(rng, Wr, Hr, pos=rng.uniform(-0.5, 0.5, 3), target=rng.uniform(-2, 2, 3))
        tri, l, z, uv = mesh.raster(cam, Hr, Wr, want_uv=True)
        ref, zt, stable = bf.raycast64(cam, V, F, Hr, Wr)
        m = stable
        assert np.array_equal(tri[m], ref[m]), (scene, np.argwhere((tri != ref) & m)[:5])
        hit = m & (ref >= 0)
        assert np.all(np.abs(z[hit] - zt[hit]) <= 1e-5 * zt[hit])
        # uv in the uv frame (A, B, C) = faces_uv: point = A + u (C - A) + v (B - A)
        R = cam[4:13].astype(np.float64).reshape(3, 3)
        t = cam[13:16].astype(np.float64)
        for (y, x) in np.argwhere(hit):
            T = ref[y, x]
            A, B, C = (V[mesh.faces_uv[T, k]].astype(np.float64) @ R.T + t for k in range(3))
            d = np.array([(x + 0.5 - cam[2]) / cam[0], (y + 0.5 - cam[3]) / cam[1], 1.0])
            M = np.stack([d, -(C - A), -(B - A)], 1)
            zz, u, v = np.linalg.solve(M, A)
            assert abs(u - uv[y, x, 0]) <= 1e-4 and abs(v - uv[y, x, 1]) <= 1e-4
            su, sv = s * u, s * v
            fr = [su - math.floor(su), sv - math.floor(sv)]
            if min(min(f, 1 - f) for f in fr) < 1e-3 or abs(fr[0] + fr[1] - 1) < 1e-3 or \
                    abs(su + sv - s) < 1e-3 or u < 1e-3 or v < 1e-3:
                continue
            assert l[y, x] - mesh.off[T] == oracle.texel_id(s, scheme, np.float32(u), np.float32(v))
            n_checked += 1
    assert n_checked > 1000


def test_watertight_floor_crossing_near_plane_and_offscreen():
    """A large planar floor grid (interior vertices moved within the plane, so
    no fold-overs) seen from 0.5 m above, extending behind the
    camera (near-plane clipping) and beyond the guard band: every pixel is
    covered at most once, and exactly once where the binary64 ray cast hits
    the floor stably."""
    rng = np.random.default_rng(7)
    n = 24
    xs = np.linspace(-30, 30, n + 1)
    P = np.zeros((n + 1, n + 1, 3))
    P[..., 0], P[..., 1] = np.meshgrid(xs, xs, indexing="ij")
    P[1:-1, 1:-1, :2] += rng.uniform(-0.4, 0.4, (n - 1, n - 1, 2))
    V = P.reshape(-1, 3).astype(np.float32)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    F = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = idx[i, j], idx[i + 1, j], idx[i + 1, j + 1], idx[i, j + 1]
            F += [[a, b, c], [a, c, d]]
    F = np.array(F, np.int32)
    mesh = oracle.Mesh(V, F, s=2, scheme=oracle.SPLIT)
    for k in range(3):
        cam = _random_cam(rng, 96, 72, pos=np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), 0.5]),
                          target=np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), -0.3]))
        cnt = mesh.coverage_count(cam, 72, 96)
        assert cnt.max() <= 1
        ref, _, stable = bf.raycast64(cam, V, F, 72, 96)
        sel = stable & (ref >= 0)
        assert sel.sum() > 1000
        assert (cnt[sel] == 1).all()
        tri, _, _ = mesh.raster(cam, 72, 96)
        assert np.array_equal(tri[stable], ref[stable])


def test_uv_origin_is_closest_to_right_angle():
    """Section 3.1: the uv origin is the vertex whose interior angle is
    closest to 90 degrees (checked with binary64 arccos; near-ties skipped)."""
    rng = np.random.default_rng(2)
    V = rng.normal(size=(3000, 3)).astype(np.float32)
    F = np.arange(3000, dtype=np.int32).reshape(-1, 3)
    mesh = oracle.Mesh(V, F)
    checked = 0
    for t in range(F.shape[0]):
        P = V[F[t]].astype(np.float64)
        ang = []
        for m in range(3):
            a = P[(m + 1) % 3] - P[m]
            b = P[(m + 2) % 3] - P[m]
            ang.append(abs(math.degrees(math.acos(a @ b / np.linalg.norm(a) / np.linalg.norm(b))) - 90))
        o = int(np.argmin(ang))
        srt = sorted(ang)
        if srt[1] - srt[0] < 1e-3:
            continue
        # origin first, then the input cyclic order (uv (0,1) then (1,0))
        assert list(mesh.faces_uv[t]) == [F[t, o], F[t, (o + 1) % 3], F[t, (o + 2) % 3]]
        checked += 1
    assert checked > 900
    # right triangle: the right-angle vertex is the origin
    V2 = np.array([[1, 0, 0], [0, 0, 0], [0, 1, 0]], np.float32)
    m2 = oracle.Mesh(V2, np.array([[0, 1, 2]], np.int32))
    assert list(m2.faces_uv[0]) == [1, 2, 0]


def test_offsets_and_invalid_faces():
    V = np.zeros((4, 3), np.float32)
    F = np.array([[0, 1, 2], [1, 2, 3], [0, 2, 3]], np.int32)
    m = oracle.Mesh(V, F, s_face=np.array([1, 3, 2]), scheme=oracle.SQUARE)
    assert list(m.off) == [0, 1, 7, 10]
    m = oracle.Mesh(V, F, s_face=np.array([1, 3, 2]), scheme=oracle.SPLIT)
    assert list(m.off) == [0, 1, 10, 14]
    with pytest.raises(ValueError):
        oracle.Mesh(V, np.array([[0, 1, 4]], np.int32))
    with pytest.raises(ValueError):
        oracle.Mesh(V, np.array([[0, 1, -1]], np.int32))
    with pytest.raises(ValueError):
        oracle.Mesh(V, F, s=0)
