"""Pins of four oracle rules that the other oracle tests do not reach, each
checked against a reference that shares nothing with the oracle:

* the guard-band clip planes (renderer, Section 3.3.1: clipped polygons stay
  within |px|, |py| <= 2^20) against an exact-rational Sutherland-Hodgman
  clip, projection and round-half-even snap;
* the crossing rule of the clip (a crossing is computed from the edge's
  inside end, so two triangles that traverse a near-clipped edge in opposite
  directions produce the same vertex bits: the renderer stays watertight);
* argmax ties in the normalisation (Section 3.2.1: the argmax is the texel's
  class; ties go to the lowest class index) against numpy's argmax;
* bfloat16 rounding of the learned weight's hidden layer against a binary64
  evaluation with torch's bfloat16 casts.

CPU only."""
from fractions import Fraction

import numpy as np
import torch

import oracle
from oracle import mlp
from tests import bruteforce as bf

G = 2 ** 20
Z_NEAR = np.float32(0.05)


def _cam(fx, fy, cx, cy):
    """Pinhole camera at the origin looking down +z (identity rotation): the
    camera-space corners equal the world corners exactly."""
    return np.array([fx, fy, cx, cy, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def _exact_clip(cam, pts):
    """Sutherland-Hodgman over the near plane and the four guard planes in
    that order, in exact rational arithmetic; points on a plane are inside."""
    fx, fy, cx, cy = (Fraction(float(v)) for v in cam[:4])
    zn = Fraction(float(Z_NEAR))
    planes = (
        lambda p: p[2] - zn,
        lambda p: (G - cx) * p[2] - fx * p[0],
        lambda p: (G + cx) * p[2] + fx * p[0],
        lambda p: (G - cy) * p[2] - fy * p[1],
        lambda p: (G + cy) * p[2] + fy * p[1],
    )
    poly = [tuple(Fraction(float(v)) for v in p) for p in pts]
    for d in planes:
        if not poly:
            break
        out = []
        n = len(poly)
        for i in range(n):
            a, b = poly[i], poly[(i + 1) % n]
            da, db = d(a), d(b)
            if da >= 0:
                out.append(a)
            if (da >= 0) != (db >= 0):
                al = da / (da - db)
                out.append(tuple(a[k] + al * (b[k] - a[k]) for k in range(3)))
        poly = out
    return poly


def _exact_snap(cam, p):
    fx, fy, cx, cy = (Fraction(float(v)) for v in cam[:4])
    px = fx * p[0] / p[2] + cx
    py = fy * p[1] / p[2] + cy
    return round(px * 256), round(py * 256)       # Fractions round half to even


def _fan_polygon(fan):
    """Polygon (v0, v1, ..., vn-1) of a fan of sub-triangles (v0, vi, vi+1)."""
    if len(fan) == 0:
        return []
    return [tuple(fan[0][0]), tuple(fan[0][1])] + [tuple(f[2]) for f in fan]


def test_guard_band_clip_against_exact_rationals():
    """Triangles reaching far beyond the image on every side (one corner at
    a few cm of depth, some behind the near plane) project beyond
    |px|, |py| > 2^20: the oracle's clipped, snapped polygon equals the exact
    rational clip vertex by vertex (to the binary32 rounding of a coordinate
    near 2^28 sub-pixel units), its guard vertices sit on |px| = 2^20 or
    |py| = 2^20, and the pixels inside the image agree with a binary64 ray
    cast of the unclipped triangles."""
    rng = np.random.default_rng(2024)
    cam = _cam(64, 64, 37, 29)           # cx != cy != 0: a sign slip in any guard plane moves it by 58-74 px
    H, W = 48, 64
    hits = {1: 0, 2: 0, 3: 0, 4: 0}
    tris = []
    for side in (1, 2, 3, 4):
        for _ in range(12):
            far = np.zeros(3)
            a = rng.uniform(1500.0, 20000.0)
            far[0] = a if side == 1 else (-a if side == 2 else rng.uniform(-1, 1))
            far[1] = a if side == 3 else (-a if side == 4 else rng.uniform(-1, 1))
            far[2] = rng.uniform(-0.5, 0.25)  # behind the near plane, or just in front of it
            p0 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(1, 3)])
            p1 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(1, 3)])
            tris.append(np.stack([p0, far, p1]).astype(np.float32))
    V = np.concatenate(tris).astype(np.float32)
    F = np.arange(V.shape[0], dtype=np.int32).reshape(-1, 3)
    mesh = oracle.Mesh(V, F, s=1, scheme=oracle.SPLIT)
    for t in range(F.shape[0]):
        corners = [V[mesh.faces_uv[t, m]] for m in range(3)]
        ex = _exact_clip(cam, corners)
        got = _fan_polygon(mesh.snapped_fan(t, cam))
        want = [_exact_snap(cam, p) for p in ex]
        assert len(got) == len(want), (t, got, want)
        for (gx, gy), (wx, wy) in zip(got, want):
            assert abs(gx - wx) <= 2 + abs(wx) / 2 ** 19, (t, gx, wx)
            assert abs(gy - wy) <= 2 + abs(wy) / 2 ** 19, (t, gy, wy)
        fx, fy, cx, cy = (Fraction(float(v)) for v in cam[:4])
        for p in ex:
            px = fx * p[0] / p[2] + cx
            py = fy * p[1] / p[2] + cy
            assert abs(px) <= G and abs(py) <= G
            for k, on in ((1, px == G), (2, px == -G), (3, py == G), (4, py == -G)):
                hits[k] += on
        for gx, gy in got:
            assert abs(gx) <= 256 * G + 2 ** 10 and abs(gy) <= 256 * G + 2 ** 10
    assert all(v > 0 for v in hits.values()), hits      # every guard plane clipped something
    tri, _, _ = mesh.raster(cam, H, W)
    ref, _, stable = bf.raycast64(cam, V, F, H, W)
    assert stable.sum() > 0.5 * H * W
    assert np.array_equal(tri[stable], ref[stable])


def test_near_clipped_shared_edge_same_bits_both_ways():
    """Two triangles share an edge P-Q that crosses the near plane and
    traverse it in opposite directions (P->Q and Q->P).  The crossing vertex
    each clip produces on that edge has identical binary32 bits, and the pair
    covers every pixel along the shared edge exactly once."""
    rng = np.random.default_rng(99)
    cam = _cam(64, 64, 32, 24)
    for trial in range(3000):
        P = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.3, 3.0)], np.float32)
        Q = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-2.0, 0.0)], np.float32)
        R1 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.3, 3.0)], np.float32)
        R2 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.3, 3.0)], np.float32)
        p1 = oracle.clip_triangle(cam, P, Q, R1, z_near=Z_NEAR)
        p2 = oracle.clip_triangle(cam, Q, P, R2, z_near=Z_NEAR)
        Pd, Qd = P.astype(np.float64), Q.astype(np.float64)
        dP, dQ = Pd[2] - float(Z_NEAR), Qd[2] - float(Z_NEAR)
        X = Pd + dP / (dP - dQ) * (Qd - Pd)          # the crossing, binary64
        c1 = p1[np.argmin(np.abs(p1.astype(np.float64) - X).sum(1))]
        c2 = p2[np.argmin(np.abs(p2.astype(np.float64) - X).sum(1))]
        assert np.abs(c1 - X).max() <= 1e-5 * (1 + np.abs(X).max()), (trial, c1, X)
        assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32)), (trial, c1, c2)
    # coverage along a shared near-clipped edge, on the two sides of it
    H, W = 72, 96
    cam = _cam(80, 80, 48, 36)
    for trial in range(12):
        P = np.array([rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), rng.uniform(0.5, 1.5)], np.float32)
        Q = np.array([rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), rng.uniform(-1.0, -0.1)], np.float32)
        # R2 mirrors R1 through the edge's midpoint: one plane, R1 and R2 on
        # opposite sides of P-Q, so the two triangles never overlap on screen
        R1 = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6), rng.uniform(0.6, 1.2)], np.float32)
        R2 = (P + Q - R1).astype(np.float32)
        V = np.stack([P, Q, R1, R2]).astype(np.float32)
        F = np.array([[0, 1, 2], [1, 0, 3]], np.int32)
        mesh = oracle.Mesh(V, F)
        cnt = mesh.coverage_count(cam, H, W)
        assert cnt.max() <= 1, trial
        ref, _, stable = bf.raycast64(cam, V, F, H, W)
        sel = stable & (ref >= 0)
        assert sel.sum() > 200
        assert (cnt[sel] == 1).all(), trial


def test_argmax_ties_go_to_the_lowest_class():
    """Rows with two or three equal maxima: the label is the first maximal
    class (numpy's argmax) for SUM and MAXSUM rows and for the log-domain
    rows of MUL; and through fusion, two observations splitting their mass
    equally between two classes give the lower class."""
    rng = np.random.default_rng(5)
    n, c = 400, 11
    A = rng.integers(0, 64, (n, c)).astype(np.float64) / 64.0
    for r in range(n):
        k = 2 + r % 2
        pos = np.sort(rng.choice(c, k, replace=False))
        A[r, pos] = A[r].max() + 1.0
    W = np.ones(n)
    for agg in (oracle.AGG_SUM, oracle.AGG_MAXSUM):
        _, lab = oracle.finalize(A, W, aggregator=agg)
        assert np.array_equal(lab, A.argmax(1).astype(np.uint8))
    L = -A                                   # log-domain sums: maxima of -A are the minima of A
    Lt = L.copy()
    for r in range(n):
        pos = np.sort(rng.choice(c, 2, replace=False))
        Lt[r, pos] = Lt[r].max() + 0.5
    _, lab = oracle.finalize(Lt, W, aggregator=oracle.AGG_MUL)
    assert np.array_equal(lab, Lt.argmax(1).astype(np.uint8))
    # fusion: one texel seen by two pixels whose sums tie on classes 0 and 2
    l = np.zeros((1, 1, 2), np.int32)
    p = np.zeros((1, 4, 1, 2), np.float32)
    p[0, :, 0, 0] = [0.25, 0.0, 0.5, 0.25]
    p[0, :, 0, 1] = [0.5, 0.25, 0.25, 0.0]
    A2, W2 = oracle.fuse(1, 4, l, p)
    assert A2[0, 0] == A2[0, 2] == 0.75
    _, lab2 = oracle.finalize(A2, W2)
    assert lab2[0] == 0


def _q(x):
    """binary64 -> binary32 -> bfloat16 (round to nearest even), as binary64."""
    return torch.from_numpy(np.asarray(x, np.float64).astype(np.float32)).to(torch.bfloat16).double().numpy()


def test_bf16_forward_on_values_that_round():
    """Random weights and features that are not bfloat16 values: the oracle's
    forward pass equals a binary64 evaluation that rounds the weights, the
    features and the first hidden layer to bfloat16 with torch's cast."""
    rng = np.random.default_rng(31)
    NI, NH = 8, 64
    p = rng.normal(0, 0.5, mlp.nparam()).astype(np.float32)
    phi = rng.random((4000, NI)).astype(np.float32)
    assert (_q(phi) != phi).mean() > 0.9 and (_q(p) != p).mean() > 0.9
    o = 0
    W1 = p[o:o + NH * NI].reshape(NH, NI); o += NH * NI
    b1 = p[o:o + NH].astype(np.float64); o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH].astype(np.float64); o += NH
    w3 = p[o:o + NH]; o += NH
    b3 = float(p[o])
    h1 = np.maximum(_q(phi) @ _q(W1).T + b1, 0.0)
    assert (_q(h1) != h1).mean() > 0.5                         # the rounding of h1 is exercised
    h2 = np.maximum(_q(h1) @ _q(W2).T + b2, 0.0)
    ref = 1.0 / (1.0 + np.exp(-(h2 @ _q(w3) + b3)))
    got = mlp.forward(p, phi, round_mode=1)
    d = np.abs(got - ref)
    assert (d <= 1e-12).mean() >= 0.999, np.quantile(d, [0.5, 0.99])
    assert d.max() <= 1e-3
    # and the rounded network is measurably not the plain one on these inputs
    plain = mlp.forward(p, phi, round_mode=0)
    assert (np.abs(plain - ref) > 1e-6).mean() > 0.5
