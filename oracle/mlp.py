"""Front end of the learned-weight oracle (``mlp_oracle.c``); test
infrastructure only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _c, _ptr, lib as _lib

_p, _i32, _i64, _f32, _f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
NI, NH = 8, 64


def _L():
    L = _lib()
    if not getattr(L, "_mlp_declared", False):
        L.om_nparam.restype = _i32
        L.om_bf16.restype = _f32
        L.om_bf16.argtypes = [_f32]
        L.om_forward.restype = None
        L.om_forward.argtypes = [_p, _p, _i64, _i32, _p]
        L.om_loss_grad.restype = _f64
        L.om_loss_grad.argtypes = [_p, _p, _p, _i64, _i32, _p]
        L.om_adam.restype = None
        L.om_adam.argtypes = [_p, _p, _p, _p, _i64, _f64, _f64, _f64, _f64, _i32]
        L.om_frame_features.restype = _i64
        L.om_frame_features.argtypes = [_p, _i64, _p, _p, _p, _i32, _i64, _p, _f32, _i32, _i32, _p, _i64, _i64, _i64,
                                        _i32, _p, _p, _p, _p, _p]
        L._mlp_declared = True
    return L


def nparam() -> int:
    return int(_L().om_nparam())


def bf16(x: float) -> float:
    return float(_L().om_bf16(float(x)))


def forward(params, phi, round_mode=1):
    params = _c(params, np.float32)
    phi = _c(phi, np.float32)
    out = np.empty(phi.shape[0], np.float64)
    _L().om_forward(_ptr(params), _ptr(phi), phi.shape[0], int(round_mode), _ptr(out))
    return out


def loss_grad(params, phi, target, round_mode=1):
    params = _c(params, np.float32)
    phi = _c(phi, np.float32)
    target = _c(target, np.float32)
    g = np.empty(nparam(), np.float64)
    loss = _L().om_loss_grad(_ptr(params), _ptr(phi), _ptr(target), phi.shape[0], int(round_mode), _ptr(g))
    return float(loss), g


def adam(params, m, v, grad, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    params = np.ascontiguousarray(params, np.float32)
    _L().om_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(_c(grad, np.float64)), params.size, lr, b1, b2, eps, int(t))
    return params


def frame_features(mesh, cam16, H, W, probs_chw, valid=None, labels=None, z_near=0.05):
    """phi [N,8], target [N] (or None), pixel index [N] of one frame."""
    probs_chw = np.asarray(probs_chw, np.float32)
    c = probs_chw.shape[0]
    cap = H * W
    phi = np.empty((cap, NI), np.float32)
    tgt = np.empty(cap, np.float32) if labels is not None else None
    pix = np.empty(cap, np.int32)
    st = [s // 4 for s in probs_chw.strides]
    n = _L().om_frame_features(_ptr(mesh.vertices), mesh.n_faces, _ptr(mesh.faces_uv), _ptr(mesh.s_face),
                               _ptr(mesh.off), mesh.scheme, mesh.n_texels, _ptr(_c(cam16, np.float32)), float(z_near),
                               H, W, probs_chw.ctypes.data_as(_p), st[0], st[1], st[2], c,
                               _ptr(None if valid is None else _c(valid, np.uint8)),
                               _ptr(None if labels is None else _c(labels, np.uint8)), _ptr(phi), _ptr(tgt), _ptr(pix))
    if n < 0:
        raise MemoryError("oracle features failed")
    return phi[:n], (tgt[:n] if tgt is not None else None), pix[:n]
