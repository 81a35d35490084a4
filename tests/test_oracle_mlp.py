"""Pins of the learned-weight oracle (MLP forward/backward, Adam, features,
bfloat16 rounding).  CPU only."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp

RNG = np.random.default_rng(77)


def _params(scale=0.3):
    return (RNG.normal(0, scale, mlp.nparam())).astype(np.float32)


def test_bf16_rounding_matches_library_cast():
    x = np.concatenate([RNG.normal(0, 1, 20000), RNG.normal(0, 1e-30, 2000), RNG.normal(0, 1e30, 2000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    mine = np.array([mlp.bf16(v) for v in x], np.float32)
    assert np.array_equal(mine.view(np.uint32), ref.view(np.uint32))


def test_zero_network_and_bce_value():
    p = np.zeros(mlp.nparam(), np.float32)
    phi = RNG.random((10, 8)).astype(np.float32)
    assert np.allclose(mlp.forward(p, phi), 0.5)
    p[-1] = 2.0  # b3
    assert np.allclose(mlp.forward(p, phi), 1 / (1 + math.exp(-2.0)))
    p[-1] = 0.0
    loss, g = mlp.loss_grad(p, phi, np.ones(10, np.float32))
    assert abs(loss - math.log(2.0)) < 1e-12
    assert abs(g[-1] - (0.5 - 1.0)) < 1e-12        # d loss / d b3 = mean(sigmoid - y)


def test_hand_built_network():
    """w = sigmoid(2 * relu(phi_3 - 0.5) - 1) built from explicit weights."""
    p = np.zeros(mlp.nparam(), np.float32)
    NI, NH = 8, 64
    W1, b1 = 0, NH * NI
    W2, b2 = b1 + NH, b1 + NH + NH * NH
    w3, b3 = b2 + NH, b2 + 2 * NH
    p[W1 + 0 * NI + 3] = 1.0
    p[b1 + 0] = -0.5
    p[W2 + 0 * NH + 0] = 1.0
    p[w3 + 0] = 2.0
    p[b3] = -1.0
    phi = np.zeros((5, 8), np.float32)
    phi[:, 3] = [0.0, 0.5, 0.75, 1.0, 2.0]
    exp = 1 / (1 + np.exp(-(2 * np.maximum(phi[:, 3].astype(np.float64) - 0.5, 0) - 1)))
    assert np.allclose(mlp.forward(p, phi, round_mode=0), exp, rtol=1e-12)
    assert np.allclose(mlp.forward(p, phi, round_mode=1), exp, rtol=1e-12)   # all values exact in bf16


def test_gradients_by_central_differences():
    p = _params()
    phi = RNG.random((40, 8)).astype(np.float32)
    y = (RNG.random(40) > 0.5).astype(np.float32)
    _, g = mlp.loss_grad(p, phi, y, round_mode=0)
    idx = np.concatenate([RNG.choice(mlp.nparam() - 1, 300, replace=False), [mlp.nparam() - 1]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(float(p[i])))   # small: no ReLU kink is crossed
        pp = p.astype(np.float64).copy()
        # the oracle takes binary32 parameters: differentiate along a step that
        # is exactly representable
        a = p.copy(); a[i] = np.float32(p[i] + h)
        b = p.copy(); b[i] = np.float32(p[i] - h)
        ha = float(a[i]) - float(p[i]); hb = float(p[i]) - float(b[i])
        la, _ = mlp.loss_grad(a, phi, y, round_mode=0)
        lb, _ = mlp.loss_grad(b, phi, y, round_mode=0)
        fd = (la - lb) / (ha + hb)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])
    del pp


def test_adam_first_step():
    p = _params()
    g = RNG.normal(0, 1, mlp.nparam())
    m = np.zeros(mlp.nparam()); v = np.zeros(mlp.nparam())
    p2 = mlp.adam(p.copy(), m, v, g, lr=1e-3, t=1)
    # first bias-corrected step is lr * g / (|g| + eps)
    exp = (p.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)).astype(np.float32)
    assert np.array_equal(p2, exp)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_feature_closed_forms():
    L = mlp._L()
    import ctypes as C
    out = np.empty(8)
    c = 4

    def feats(rx, ry, n, z, u, v, p, cnt, x, y, cx, cy):
        pa = np.asarray(p, np.float64)
        na = np.asarray(n, np.float64)
        L.om_features.restype = None
        L.om_features.argtypes = [C.c_double, C.c_double, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                  C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.om_features(rx, ry, na.ctypes.data, z, u, v, pa.ctypes.data, len(p), cnt, x, y, cx, cy, out.ctypes.data)
        return out.copy()

    # head-on ray through the image centre, uniform distribution, centroid, one pixel
    f = feats(0.0, 0.0, [0, 0, -3.0], 1.0, 1 / 3, 1 / 3, [0.25] * 4, 1, 49.5, 29.5, 50, 30)
    assert np.allclose(f, [1.0, 0.5, 1.0, 0.25, 0.0, 1.0, 0.0, 0.0])
    # grazing ray (normal perpendicular to it), one-hot, on an edge, 64 pixels, image corner
    f = feats(1.0, 0.0, [0, 1.0, 0], 3.0, 0.0, 0.5, [0, 1, 0, 0], 64, -0.5, -0.5, 50, 30)
    assert np.allclose(f, [0.0, 0.75, 0.0, 1.0, 1.0, 0.0, 1.0, 1.0])
    # 45 degrees, two tied maxima, 4096 pixels (clamped at 2)
    f = feats(1.0, 0.0, [0, 0, 1.0], 1.0, 0.2, 0.2, [0.4, 0.4, 0.2, 0.0], 4096, 0, 0, 0.5, 0.5)
    assert abs(f[0] - math.sqrt(0.5)) < 1e-12 and f[3] == 0.4 and f[4] == 0.0 and f[6] == 2.0
    ent = -(2 * 0.4 * math.log(0.4) + 0.2 * math.log(0.2)) / math.log(4)
    assert abs(f[2] - ent) < 1e-12
