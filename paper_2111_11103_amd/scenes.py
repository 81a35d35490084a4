"""Seeded synthetic scenes and per-pixel class distributions.

This module only *generates inputs*: a triangle mesh of a procedural room,
camera poses, a ground-truth class per pixel (by an analytic ray cast against
the room's axis-aligned boxes, not by the mesh rasterizer), and the synthetic
"segmentation network" output p_k = softmax(logits).  It contains none of the
label-fusion arithmetic; both the GPU path and the CPU oracle consume the
bytes it produces.

The workloads stand in for the paper's ScanNet v2 meshes with ESANet
predictions over the 40 NYUv2 classes (Section 4.1): those datasets and
weights are not used; the recipe is

* room: an axis-aligned box [0,Lx]x[0,Ly]x[0,Lz] (z up), every face a regular
  quad grid split into two triangles per quad, vertices shared inside a face;
* obstacles: axis-aligned boxes standing on the floor, tessellated the same
  way; one class per object (floor, ceiling, 4 walls, then one per box),
  taken modulo the number of classes;
* cameras: pinhole, fx = fy = 0.8 W, cx = W/2, cy = H/2, OpenCV axes
  (x right, y down, z forward); extrinsics map world to camera,
  X_c = R X_w + t;
* logits_j = m [j = l'] + eps_j, eps ~ N(0, sigma^2) with sigma the standard
  deviation; l' is the ground truth except inside random discs covering a
  target fraction of the frame, where it is shifted by a random non-zero
  class offset (always wrong); an optional Bernoulli mask marks pixels with
  no depth (valid = 0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "Box", "room_scene", "circle_cameras", "random_walk_cameras",
    "camera_matrix", "ground_truth", "make_probs", "quantize_fp8", "frame_inputs",
    "config1", "config2",
]


@dataclass
class Box:
    lo: np.ndarray  # (3,) float64
    hi: np.ndarray  # (3,) float64
    cls: int        # class of every face (obstacle) or -1 for the room (per-face classes)


@dataclass
class Scene:
    vertices: np.ndarray          # [V,3] float32 world coordinates
    faces: np.ndarray             # [T,3] int32 vertex indices
    face_class: np.ndarray        # [T] int32 ground-truth class of every triangle
    room: Box                     # room box (interior), classes 0..5 per face
    boxes: list = field(default_factory=list)  # obstacle boxes
    n_classes: int = 13

    @property
    def n_faces(self) -> int:
        return int(self.faces.shape[0])


# --------------------------------------------------------------------------- mesh

def _grid_face(origin, du, dv, nu, nv):
    """Vertices [(nu+1)(nv+1),3] and triangles [2 nu nv,3] of a planar quad grid."""
    iu = np.arange(nu + 1, dtype=np.float64)
    iv = np.arange(nv + 1, dtype=np.float64)
    U, Vv = np.meshgrid(iu / nu, iv / nv, indexing="ij")
    pts = origin[None, None, :] + U[..., None] * du[None, None, :] + Vv[..., None] * dv[None, None, :]
    pts = pts.reshape(-1, 3)
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    tris = np.empty((2 * nu * nv, 3), dtype=np.int64)
    tris[0::2] = np.stack([a, b, c], 1)
    tris[1::2] = np.stack([a, c, d], 1)
    return pts, tris


def _box_faces(lo, hi):
    """Six faces of an axis-aligned box as (origin, du, dv, extent_u, extent_v)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    ex = hi - lo
    X = np.array([ex[0], 0, 0]); Y = np.array([0, ex[1], 0]); Z = np.array([0, 0, ex[2]])
    return [
        (lo.copy(), X, Y),                        # z = lo (floor / bottom)
        (lo + Z, X, Y),                           # z = hi (ceiling / top)
        (lo.copy(), X, Z),                        # y = lo
        (lo + Y, X, Z),                           # y = hi
        (lo.copy(), Y, Z),                        # x = lo
        (lo + X, Y, Z),                           # x = hi
    ]


def _place_boxes(rng, room_hi, n_boxes, edge_lo, edge_hi, margin=0.2):
    boxes = []
    tries = 0
    while len(boxes) < n_boxes:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place boxes")
        e = rng.uniform(edge_lo, edge_hi, size=3)
        x0 = rng.uniform(margin, room_hi[0] - margin - e[0])
        y0 = rng.uniform(margin, room_hi[1] - margin - e[1])
        lo = np.array([x0, y0, 0.0])
        hi = lo + e
        ok = True
        for b in boxes:
            if (lo[0] < b.hi[0] + 0.05 and b.lo[0] < hi[0] + 0.05 and
                    lo[1] < b.hi[1] + 0.05 and b.lo[1] < hi[1] + 0.05):
                ok = False
                break
        if ok:
            boxes.append(Box(lo, hi, -1))
    return boxes


def room_scene(seed: int = 0, room=(6.0, 5.0, 3.0), n_boxes: int = 6, n_classes: int = 13,
               cell: float | None = None, room_grid: int | None = 13, box_grid: int | None = 1,
               edge=(0.3, 1.2)) -> Scene:
    """Procedural room plus obstacle boxes.

    With ``cell`` set, every face is tessellated into quads of side about
    ``cell`` metres (uniform triangle density); otherwise room faces use a
    ``room_grid`` x ``room_grid`` grid and box faces a ``box_grid`` grid.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    room_hi = np.asarray(room, np.float64)
    boxes = _place_boxes(rng, room_hi, n_boxes, edge[0], edge[1])
    verts, tris, fcls = [], [], []
    nv_total = 0
    objs = []
    for fi, (org, du, dv) in enumerate(_box_faces(np.zeros(3), room_hi)):
        objs.append((org, du, dv, fi % n_classes, room_grid))
    for bi, b in enumerate(boxes):
        b.cls = (6 + bi) % n_classes
        for (org, du, dv) in _box_faces(b.lo, b.hi):
            objs.append((org, du, dv, b.cls, box_grid))
    for org, du, dv, cls, g in objs:
        if cell is not None:
            nu = max(1, int(round(np.linalg.norm(du) / cell)))
            nvv = max(1, int(round(np.linalg.norm(dv) / cell)))
        else:
            nu = nvv = int(g)
        p, t = _grid_face(org, du, dv, nu, nvv)
        verts.append(p)
        tris.append(t + nv_total)
        fcls.append(np.full(t.shape[0], cls, np.int32))
        nv_total += p.shape[0]
    V = np.concatenate(verts).astype(np.float32)
    F = np.concatenate(tris).astype(np.int32)
    C = np.concatenate(fcls).astype(np.int32)
    return Scene(vertices=V, faces=F, face_class=C, room=Box(np.zeros(3), room_hi, -1),
                 boxes=boxes, n_classes=n_classes)


def cell_for_triangles(room, boxes_area: float, target_tris: int) -> float:
    """Quad side length that gives about ``target_tris`` triangles."""
    lx, ly, lz = room
    area = 2 * (lx * ly + lx * lz + ly * lz) + boxes_area
    return math.sqrt(2.0 * area / target_tris)


# --------------------------------------------------------------------------- cameras

def camera_matrix(pos, target, W: int, H: int, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera record [16] float32 = fx, fy, cx, cy, R (row-major, world->camera), t."""
    pos = np.asarray(pos, np.float64)
    f = np.asarray(target, np.float64) - pos
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0)
    t = -R @ pos
    fx = fy = 0.8 * W
    rec = np.concatenate([[fx, fy, W / 2.0, H / 2.0], R.ravel(), t]).astype(np.float32)
    return rec


def circle_cameras(scene: Scene, n_frames: int, W: int, H: int, radius=1.5, height=1.5,
                   target_height=0.75) -> np.ndarray:
    cx, cy = scene.room.hi[0] / 2, scene.room.hi[1] / 2
    cams = []
    for f in range(n_frames):
        th = 2 * math.pi * f / n_frames
        pos = (cx + radius * math.cos(th), cy + radius * math.sin(th), height)
        cams.append(camera_matrix(pos, (cx, cy, target_height), W, H))
    return np.stack(cams)


def random_walk_cameras(scene: Scene, n_frames: int, W: int, H: int, seed: int = 0,
                        min_dist=0.3, smooth=0.9, step=0.08) -> np.ndarray:
    """Smooth random walk: low-pass filtered Gaussian steps, slowly varying yaw/pitch."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    hi = scene.room.hi
    top = max([b.hi[2] for b in scene.boxes] + [0.0])
    zlo = max(top + min_dist, 1.2)
    zhi = hi[2] - min_dist
    pos = np.array([hi[0] / 2, hi[1] / 2, (zlo + zhi) / 2])
    vel = np.zeros(3)
    yaw = rng.uniform(0, 2 * math.pi)
    yaw_rate = 0.0
    pitch = -0.35
    cams = []
    for _ in range(n_frames):
        vel = smooth * vel + (1 - smooth) * rng.normal(0, step, 3) * np.array([1, 1, 0.3])
        pos = pos + vel
        for a in range(3):
            lo_a = min_dist if a < 2 else zlo
            hi_a = hi[a] - min_dist if a < 2 else zhi
            if pos[a] < lo_a:
                pos[a] = lo_a; vel[a] = abs(vel[a])
            if pos[a] > hi_a:
                pos[a] = hi_a; vel[a] = -abs(vel[a])
        yaw_rate = 0.95 * yaw_rate + 0.05 * rng.normal(0, 0.08)
        yaw += yaw_rate
        pitch = float(np.clip(0.97 * pitch + 0.03 * rng.normal(-0.45, 0.4), -1.0, -0.05))
        d = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
        cams.append(camera_matrix(pos, pos + d, W, H))
    return np.stack(cams)


# --------------------------------------------------------------------------- ground truth

def ground_truth(scene: Scene, cams, H: int, W: int, device="cpu", geometry=False):
    """Class of the first surface hit by each pixel-centre ray, by an analytic
    ray cast against the room's boxes.  Returns int64 [F,H,W]; with
    ``geometry`` also the depth z and |cos| of the viewing angle of the hit
    (float32 [F,H,W] each)."""
    import torch
    cams_t = torch.as_tensor(np.asarray(cams, np.float64), device=device)
    F = cams_t.shape[0]
    fx, fy, cx, cy = cams_t[:, 0], cams_t[:, 1], cams_t[:, 2], cams_t[:, 3]
    R = cams_t[:, 4:13].reshape(F, 3, 3)
    t = cams_t[:, 13:16]
    xs = torch.arange(W, device=device, dtype=torch.float64) + 0.5
    ys = torch.arange(H, device=device, dtype=torch.float64) + 0.5
    dx = (xs[None, :] - cx[:, None]) / fx[:, None]            # [F,W]
    dy = (ys[None, :] - cy[:, None]) / fy[:, None]            # [F,H]
    dcam = torch.stack([dx[:, None, :].expand(F, H, W), dy[:, :, None].expand(F, H, W),
                        torch.ones(F, H, W, device=device, dtype=torch.float64)], -1)
    Rt = R.transpose(1, 2)
    d = torch.einsum("fij,fhwj->fhwi", Rt, dcam)              # world ray directions
    o = -(Rt @ t[:, :, None])[:, :, 0]                        # camera centres
    o = o[:, None, None, :].expand_as(d)
    big = torch.tensor(float("inf"), device=device, dtype=torch.float64)
    # room: exit distance through the interior; face index -> class
    lo = torch.as_tensor(scene.room.lo, device=device)
    hi = torch.as_tensor(scene.room.hi, device=device)
    with np.errstate(divide="ignore"):
        inv = 1.0 / d
    t_lo = (lo - o) * inv
    t_hi = (hi - o) * inv
    t_exit_axis = torch.where(d > 0, t_hi, torch.where(d < 0, t_lo, big))
    best_t, axis = t_exit_axis.min(-1)
    pos_side = torch.gather(d, -1, axis[..., None])[..., 0] > 0
    # face order of room_scene: z-lo, z-hi, y-lo, y-hi, x-lo, x-hi
    face_of_axis = torch.tensor([[4, 5], [2, 3], [0, 1]], device=device)
    face = face_of_axis[axis, pos_side.long()]
    cls = face % scene.n_classes
    hit_axis = axis.clone()
    for b in scene.boxes:
        blo = torch.as_tensor(b.lo, device=device)
        bhi = torch.as_tensor(b.hi, device=device)
        t1 = (blo - o) * inv
        t2 = (bhi - o) * inv
        tmin = torch.minimum(t1, t2)
        tmax = torch.maximum(t1, t2)
        tmin = torch.where(torch.isnan(tmin), -big, tmin)
        tmax = torch.where(torch.isnan(tmax), big, tmax)
        tn = tmin.max(-1).values
        tf = tmax.min(-1).values
        hit = (tn <= tf) & (tn > 0) & (tn < best_t)
        best_t = torch.where(hit, tn, best_t)
        cls = torch.where(hit, torch.full_like(cls, b.cls), cls)
        hit_axis = torch.where(hit, tmin.argmax(-1), hit_axis)
    if not geometry:
        return cls
    # the camera-space ray is (dx, dy, 1), so the ray parameter is the depth
    dn = torch.gather(d, -1, hit_axis[..., None])[..., 0].abs() / d.norm(dim=-1)
    return cls, best_t.to(torch.float32), dn.to(torch.float32)


# --------------------------------------------------------------------------- probabilities

def make_probs(gt, n_classes: int, margin: float, sigma: float, blob_frac: float,
               seed: int = 0, out=None, blob_r=(0.03, 0.12), quality=None, shift_px: int = 0):
    """Synthetic network output [F,c,H,W] float32 (NCHW).

    ``gt`` is an int64 tensor [F,H,W] on the generating device.  ``out`` may be a
    preallocated float32 tensor of the right shape (filled in place).
    ``quality`` (optional float32 [F,H,W] in [0, 1]) makes the noise depend
    on the view: a pixel of quality q gets the margin * (0.5 + 0.5 q) and the
    noise sigma * (1.3 - 0.3 q), and a mislabel disc relabels only its
    pixels whose quality is below a threshold drawn from U(0.4, 0.8).
    ``shift_px`` > 0 shifts each frame's label map by an integer offset drawn
    from [-shift_px, shift_px]^2 before the noise is added.
    """
    import torch
    device = gt.device
    F, H, W = gt.shape
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1000003 + 17)
    lab = gt.clone()
    if shift_px > 0:
        # misregistration: the network sees the image under a slightly wrong
        # pose, so its labels are the ground truth moved by up to shift_px
        # pixels (edge pixels repeated)
        for f in range(F):
            d = torch.randint(-shift_px, shift_px + 1, (2,), generator=g, device=device)
            ys = (torch.arange(H, device=device) - d[1]).clamp(0, H - 1)
            xs = (torch.arange(W, device=device) - d[0]).clamp(0, W - 1)
            lab[f] = gt[f][ys][:, xs]
    yy = torch.arange(H, device=device, dtype=torch.float32)[:, None]
    xx = torch.arange(W, device=device, dtype=torch.float32)[None, :]
    mn = min(H, W)
    for f in range(F):
        covered = torch.zeros(H, W, dtype=torch.bool, device=device)
        target = blob_frac * H * W
        guard = 0
        while blob_frac > 0 and float(covered.sum()) < target and guard < 1000:
            guard += 1
            r = (blob_r[0] + (blob_r[1] - blob_r[0]) * torch.rand((), generator=g, device=device)) * mn
            cxy = torch.rand(2, generator=g, device=device) * torch.tensor([W, H], device=device, dtype=torch.float32)
            delta = torch.randint(1, n_classes, (), generator=g, device=device)
            disc = (xx + 0.5 - cxy[0]) ** 2 + (yy + 0.5 - cxy[1]) ** 2 <= r * r
            if quality is not None:
                # view-dependent mislabels: only the disc's low-quality pixels
                qt = 0.4 + 0.4 * torch.rand((), generator=g, device=device)
                disc &= quality[f].to(device) < qt
            newpix = disc & ~covered
            lab[f] = torch.where(newpix, (gt[f] + delta) % n_classes, lab[f])
            covered |= disc
    if out is None:
        out = torch.empty((F, n_classes, H, W), dtype=torch.float32, device=device)
    for f in range(F):
        logits = torch.randn((n_classes, H, W), generator=g, device=device, dtype=torch.float32)
        if quality is None:
            logits *= sigma
            add = torch.full((1, H, W), float(margin), device=device)
        else:
            q = quality[f].to(device=device, dtype=torch.float32).clamp(0.0, 1.0)
            logits *= (sigma * (1.3 - 0.3 * q))[None]
            add = (margin * (0.5 + 0.5 * q))[None]
        logits.scatter_add_(0, lab[f][None], add)
        out[f] = torch.softmax(logits, dim=0)
    return out


def quantize_fp8(probs):
    """Per-pixel scaled OCP E4M3FN codes: sigma_k = max_j p_kj / 448, q = e4m3(p / sigma).

    Returns (codes uint8 [F,c,H,W], scale float32 [F,H,W]).  Rounding is the
    library cast (round to nearest even, saturating at 448 by construction).
    """
    import torch
    scale = probs.amax(dim=1) / 448.0
    safe = torch.where(scale > 0, scale, torch.ones_like(scale))
    q = (probs / safe[:, None]).clamp(max=448.0).to(torch.float8_e4m3fn).view(torch.uint8)
    return q, scale.contiguous()


# --------------------------------------------------------------------------- workloads

@dataclass
class FrameInputs:
    scene: Scene
    cams: np.ndarray      # [F,16] float32
    H: int
    W: int
    probs: object         # torch float32 [F,c,H,W]
    valid: object         # torch uint8 [F,H,W]
    gt: object            # torch int64 [F,H,W]
    s: int = 1
    scheme: int = 1       # 0 = SQUARE (paper), 1 = SPLIT


def view_quality(z, cosv, z_ref=4.0):
    """Per-pixel view quality in [0, 1]: half from the viewing angle, half
    from the distance (1 at the camera, 1/2 at z_ref)."""
    return 0.5 * cosv + 0.5 / (1.0 + (z / z_ref) ** 2)


def frame_inputs(scene, cams, H, W, margin, sigma, blob_frac, invalid_frac, seed, device="cpu",
                 chunk=None, structured=False):
    import torch
    F = cams.shape[0]
    c = scene.n_classes
    chunk = chunk or F
    probs = torch.empty((F, c, H, W), dtype=torch.float32, device=device)
    valid = torch.empty((F, H, W), dtype=torch.uint8, device=device)
    gts = torch.empty((F, H, W), dtype=torch.int64, device=device) if F * H * W <= 50_000_000 else None
    for f0 in range(0, F, chunk):
        f1 = min(F, f0 + chunk)
        if structured:
            gt, z, cv = ground_truth(scene, cams[f0:f1], H, W, device=device, geometry=True)
            qual = view_quality(z, cv)
        else:
            gt, qual = ground_truth(scene, cams[f0:f1], H, W, device=device), None
        make_probs(gt, c, margin, sigma, blob_frac, seed=seed * 100003 + f0, out=probs[f0:f1], quality=qual,
                   shift_px=2 if structured else 0)
        g = torch.Generator(device=device)
        g.manual_seed(seed * 31337 + f0)
        if invalid_frac > 0:
            valid[f0:f1] = (torch.rand((f1 - f0, H, W), generator=g, device=device) >= invalid_frac).to(torch.uint8)
        else:
            valid[f0:f1] = 1
        if gts is not None:
            gts[f0:f1] = gt
    return probs, valid, gts


def config1(device="cpu", seed=0, n_frames=20, H=120, W=160, structured=False):
    """Plain FP32 parity workload: 2,100-triangle room, c = 13, 20 frames at
    160x120.  ``structured`` makes the probability noise depend on the view
    (see make_probs); the learned weighting trains and is evaluated on both."""
    sc = room_scene(seed=seed, room=(6.0, 5.0, 3.0), n_boxes=6, n_classes=13, room_grid=13, box_grid=1)
    cams = circle_cameras(sc, n_frames, W, H)
    probs, valid, gt = frame_inputs(sc, cams, H, W, margin=4.0, sigma=1.5, blob_frac=0.10,
                                    invalid_frac=0.0, seed=seed, device=device, structured=structured)
    return FrameInputs(sc, cams, H, W, probs, valid, gt, s=1, scheme=1)


def config2_scene(seed=0, target_tris=500_000):
    room = (8.0, 6.0, 3.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    # estimate box surface to size the grid: 20 boxes of mean edge 0.75 m
    cell = cell_for_triangles(room, 20 * 6 * 0.75 ** 2, target_tris)
    sc = room_scene(seed=seed, room=room, n_boxes=20, n_classes=40, cell=cell)
    # refine the cell size once so the count lands within 2% of the target
    T = sc.n_faces
    cell2 = cell * math.sqrt(T / target_tris)
    sc = room_scene(seed=seed, room=room, n_boxes=20, n_classes=40, cell=cell2)
    return sc


def config2(device="cpu", seed=0, n_frames=300, H=480, W=640, chunk=50, scene=None):
    """Plain FP32 at scale: ~500k-triangle room, SPLIT s = 3, c = 40, 640x480 frames."""
    sc = scene if scene is not None else config2_scene(seed)
    cams = random_walk_cameras(sc, n_frames, W, H, seed=seed)
    probs, valid, gt = frame_inputs(sc, cams, H, W, margin=3.0, sigma=2.0, blob_frac=0.15,
                                    invalid_frac=0.05, seed=seed, device=device, chunk=chunk)
    return FrameInputs(sc, cams, H, W, probs, valid, gt, s=3, scheme=1)


@dataclass
class PooledScene:
    scene: Scene
    cams: np.ndarray      # [F,16] float32, one camera per frame
    H: int
    W: int
    s: int
    pool: int             # frame f reads input frame f % pool
    probs: object         # torch float32 [pool,c,H,W]
    valid: object         # torch uint8 [pool,H,W]


def config4(device="cpu", n_scenes=16, scale=1.0, seed0=1000):
    """Batched workload: scenes i = 0..n-1 (seed 1000 + i) of uneven size,
    T_i = 50k * 40^(i/15) triangles (times ``scale``), SPLIT s_i = 1 + i mod 4,
    F_i = 100 + 60 i frames, 640x480 for even i and 1296x968 for odd i,
    c = 40.  Each scene's inputs are a pool of 16 (640x480) or 8 (1296x968)
    frames cycled by frame index, generated like the large single-scene
    workload (m = 3, sigma = 2, 15 % blobs, 5 % invalid)."""
    out = []
    for i in range(n_scenes):
        T = int(round(50_000 * 40 ** (i / 15) * scale))
        sc = config2_scene(seed=seed0 + i, target_tris=max(T, 2_000))
        s = 1 + i % 4
        F = 100 + 60 * i
        H, W = (480, 640) if i % 2 == 0 else (968, 1296)
        pool = 16 if i % 2 == 0 else 8
        cams = random_walk_cameras(sc, F, W, H, seed=seed0 + i)
        probs, valid, _ = frame_inputs(sc, cams[:pool], H, W, margin=3.0, sigma=2.0, blob_frac=0.15,
                                       invalid_frac=0.05, seed=seed0 + i, device=device)
        out.append(PooledScene(sc, cams, H, W, s, pool, probs, valid))
    return out
