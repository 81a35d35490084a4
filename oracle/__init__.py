"""CPU oracle (test infrastructure only).

Plain numpy/ctypes front end of ``semfuse_oracle.c``.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
product path never does.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "semfuse_oracle.c"), os.path.join(HERE, "mlp_oracle.c")]

_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary32 ops exactly as written: no
    contraction, no fast-math)."""
    if not force and os.path.exists(LIB):
        return LIB
    srcs = [s for s in SRC if os.path.exists(s)]
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-o", LIB + ".tmp", *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB):
                build()
            L = C.CDLL(LIB)
            _declare(L)
            _lib = L
    return _lib


_p = C.c_void_p
_i32, _i64, _f32, _f64 = C.c_int32, C.c_int64, C.c_float, C.c_double


def _declare(L):
    L.or_texel_count.restype = _i64
    L.or_texel_count.argtypes = [_i32, _i32]
    L.or_texel_id.restype = _i32
    L.or_texel_id.argtypes = [_i32, _i32, _f32, _f32]
    L.or_prepare_mesh.restype = _i32
    L.or_prepare_mesh.argtypes = [_i64, _p, _i64, _p, _p, _i32, _i32, _p, _p, _p]
    L.or_raster_frame.restype = _i32
    L.or_raster_frame.argtypes = [_p, _i64, _p, _p, _p, _i32, _p, _f32, _i32, _i32, _p, _p, _p, _p]
    L.or_coverage_count.restype = _i32
    L.or_coverage_count.argtypes = [_p, _i64, _p, _p, _f32, _i32, _i32, _p]
    L.or_snapped_fan.restype = _i32
    L.or_snapped_fan.argtypes = [_p, _p, _p, _f32, _p]
    L.or_clip_triangle.restype = _i32
    L.or_clip_triangle.argtypes = [_p, _f32, _p, _p, _p, _p]
    L.or_e4m3_decode.restype = _f64
    L.or_e4m3_decode.argtypes = [C.c_uint8]
    L.or_fuse.restype = _i32
    L.or_fuse.argtypes = [_i32, _i32, _i32, _i32, _p, _p, _p, _i32, _p, _p, _i32, _i32, _p, _i64, _p, _p]
    L.or_finalize.restype = _i32
    L.or_finalize.argtypes = [_i64, _i32, _p, _p, _i32, _p, _p]
    L.or_render.restype = _i32
    L.or_render.argtypes = [_i64, _p, _p, _p, _p]
    if hasattr(L, "om_forward"):
        from . import mlp as _mlp  # noqa: F401  (declares its own symbols)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


SQUARE, SPLIT = 0, 1
AGG_SUM, AGG_MUL, AGG_MAXSUM = 0, 1, 2
W_PIXEL, W_IMAGE, W_GIVEN = 0, 1, 2


def texel_count(s: int, scheme: int) -> int:
    return int(lib().or_texel_count(s, scheme))


def texel_id(s: int, scheme: int, u: float, v: float) -> int:
    return int(lib().or_texel_id(s, scheme, float(np.float32(u)), float(np.float32(v))))


class Mesh:
    """uv-ordered faces, texel resolution and row offsets of a mesh."""

    def __init__(self, vertices, faces, s=1, scheme=SPLIT, s_face=None):
        self.vertices = _c(vertices, np.float32)
        faces = _c(faces, np.int32)
        T = faces.shape[0]
        self.faces_uv = np.empty((T, 3), np.int32)
        self.s_face = np.empty(T, np.int32)
        self.off = np.empty(T + 1, np.int64)
        sf = None if s_face is None else _c(s_face, np.int32)
        rc = lib().or_prepare_mesh(self.vertices.shape[0], _ptr(self.vertices), T, _ptr(faces), _ptr(sf),
                                   int(s), int(scheme), _ptr(self.faces_uv), _ptr(self.s_face), _ptr(self.off))
        if rc != 0:
            raise ValueError("invalid mesh (face index out of range or s < 1)")
        self.scheme = int(scheme)
        self.n_faces = T
        self.n_texels = int(self.off[T])

    def raster(self, cam16, H, W, z_near=0.05, want_uv=False):
        """(tri, l, z[, uv]) of one frame."""
        cam = _c(cam16, np.float32)
        tri = np.empty((H, W), np.int32)
        l = np.empty((H, W), np.int32)
        z = np.empty((H, W), np.float32)
        uv = np.empty((H, W, 2), np.float32) if want_uv else None
        rc = lib().or_raster_frame(_ptr(self.vertices), self.n_faces, _ptr(self.faces_uv), _ptr(self.s_face),
                                   _ptr(self.off), self.scheme, _ptr(cam), float(z_near), H, W,
                                   _ptr(tri), _ptr(l), _ptr(z), _ptr(uv))
        if rc != 0:
            raise MemoryError("oracle raster failed")
        return (tri, l, z, uv) if want_uv else (tri, l, z)

    def raster_frames(self, cams, H, W, z_near=0.05, threads=None):
        """l and tri buffers [F,H,W] for many frames (frames in parallel)."""
        from concurrent.futures import ThreadPoolExecutor
        F = len(cams)
        tri = np.empty((F, H, W), np.int32)
        l = np.empty((F, H, W), np.int32)

        def one(f):
            t_, l_, _ = self.raster(cams[f], H, W, z_near)
            tri[f] = t_
            l[f] = l_

        n = threads or min(16, os.cpu_count() or 1)
        if n <= 1 or F == 1:
            for f in range(F):
                one(f)
        else:
            with ThreadPoolExecutor(n) as ex:
                list(ex.map(one, range(F)))
        return tri, l

    def coverage_count(self, cam16, H, W, z_near=0.05):
        cam = _c(cam16, np.float32)
        cnt = np.empty((H, W), np.int32)
        lib().or_coverage_count(_ptr(self.vertices), self.n_faces, _ptr(self.faces_uv), _ptr(cam),
                                float(z_near), H, W, _ptr(cnt))
        return cnt

    def snapped_fan(self, t, cam16, z_near=0.05):
        cam = _c(cam16, np.float32)
        out = np.zeros(36, np.int32)
        n = lib().or_snapped_fan(_ptr(self.vertices), _ptr(self.faces_uv[t]), _ptr(cam), float(z_near), _ptr(out))
        return out[: 6 * n].reshape(n, 3, 2)


def clip_triangle(cam16, A, B, C, z_near=0.05):
    """Camera-space polygon [n, 3] (binary32) of the world triangle (A, B, C),
    corners in the order given, after the near and guard-plane clip."""
    out = np.zeros((8, 3), np.float32)
    n = lib().or_clip_triangle(_ptr(_c(cam16, np.float32)), float(z_near), _ptr(_c(A, np.float32)),
                               _ptr(_c(B, np.float32)), _ptr(_c(C, np.float32)), _ptr(out))
    return out[:n].copy()


def e4m3_decode(q: int) -> float:
    return float(lib().or_e4m3_decode(int(q)))


def fuse(n_texels, c, l, probs, valid=None, weighting=W_PIXEL, aggregator=AGG_SUM, scale=None,
         wpix=None, A=None, W_sum=None):
    """Accumulate frames into (A, W_sum) in binary64.  ``probs`` is float32
    [F,c,H,W] (any strides) or uint8 E4M3 codes with ``scale`` [F,H,W]."""
    l = _c(l, np.int32)
    F, H, W = l.shape
    if A is None:
        A = np.zeros((n_texels, c), np.float64)
    if W_sum is None:
        W_sum = np.zeros(n_texels, np.float64)
    probs = np.asarray(probs)
    if probs.dtype == np.float32:
        dt = 0
    elif probs.dtype == np.uint8:
        dt = 3
        scale = _c(scale, np.float32)
    else:
        raise TypeError("probs must be float32 or uint8 (E4M3 codes)")
    strides = np.array([s // probs.itemsize for s in probs.strides], np.int64)
    v = None if valid is None else _c(valid, np.uint8)
    wp = None if wpix is None else _c(wpix, np.float32)
    rc = lib().or_fuse(F, H, W, c, _ptr(l), _ptr(v), probs.ctypes.data_as(_p), dt, _ptr(strides),
                       _ptr(scale) if dt == 3 else None, int(aggregator), int(weighting), _ptr(wp),
                       int(n_texels), _ptr(A), _ptr(W_sum))
    if rc != 0:
        raise ValueError(f"oracle fuse failed ({rc})")
    return A, W_sum


def finalize(A, W_sum=None, aggregator=AGG_SUM):
    A = _c(A, np.float64)
    n, c = A.shape
    P = np.empty_like(A)
    lab = np.empty(n, np.uint8)
    ws = None if W_sum is None else _c(W_sum, np.float64)
    lib().or_finalize(n, c, _ptr(A), _ptr(ws), int(aggregator), _ptr(P), _ptr(lab))
    return P, lab


def render(l, label, valid=None):
    l = _c(l, np.int32)
    out = np.empty(l.shape, np.uint8)
    v = None if valid is None else _c(valid, np.uint8)
    lib().or_render(l.size, _ptr(l), _ptr(v), _ptr(_c(label, np.uint8)), _ptr(out))
    return out


def triangle_max_pixels(tri_frames, n_faces):
    """a_t of Section 3.1: the most pixels triangle t wins in any one frame
    (tri_frames: per-frame triangle ids [F,H,W] from the oracle raster; -1 =
    none).  Every covered pixel counts, valid or not."""
    area = np.zeros(n_faces, np.int64)
    for f in range(tri_frames.shape[0]):
        t = tri_frames[f][tri_frames[f] >= 0]
        area = np.maximum(area, np.bincount(t, minlength=n_faces))
    return area.astype(np.int32)


def texel_resolution(area, gamma):
    """s_t = max(1, ceil(gamma * sqrt(a_t))) of Section 3.1, evaluated in
    binary32 (the paper fixes no precision; the decision is taken in the
    kernel's), capped at 4096."""
    a = np.asarray(area, np.float32)
    v = np.ceil(np.float32(gamma) * np.sqrt(a))
    return np.clip(np.maximum(v, 1), 1, 4096).astype(np.int32)
