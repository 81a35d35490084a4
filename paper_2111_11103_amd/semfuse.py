"""Python binding of the semfuse C-ABI (``include/semfuse.h``).

Argument marshalling only: tensors are passed as raw device pointers on the
current PyTorch stream, and every step runs in the library's HIP kernels.
The library must be built (``paper_2111_11103_amd/build.py``); nothing here
falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsemfuse.so")

# enums of semfuse.h
LF_OK, LF_EINVAL, LF_ESIZE, LF_EHIP, LF_ESTATE = 0, -1, -2, -3, -4
SQUARE, SPLIT = 0, 1
W_PIXEL, W_IMAGE, W_LEARNED, W_MIX = 0, 1, 2, 3
AGG_SUM, AGG_MUL, AGG_MAXSUM = 0, 1, 2
F32, BF16, F16, FP8_E4M3 = 0, 1, 2, 3
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_SORTED, SCATTER_STAGED = 0, 1, 2, 3
NOALLOC_SCRATCH_BYTES = 64 << 20   # LF_NOALLOC_SCRATCH_BYTES

_TEX_DT = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}


class SemfuseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"semfuse error {status}: {msg}")
        self.status = status


class _MeshOpts(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("s_uniform", C.c_int32), ("n_classes", C.c_int32),
                ("aggregator", C.c_int32), ("accum_dtype", C.c_int32), ("z_near", C.c_float)]


class _Tuning(C.Structure):
    _fields_ = [("tile", C.c_int32), ("gather_unroll", C.c_int32), ("small_px", C.c_int32),
                ("gather_waves", C.c_int32), ("learned_in_gather", C.c_int32)]


class _SceneJob(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("d_cams", C.c_void_p), ("F", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
                ("d_probs", C.c_void_p), ("prob_dtype", C.c_int32), ("strides", C.c_int64 * 4),
                ("d_scale", C.c_void_p), ("d_valid", C.c_void_p), ("pool", C.c_int32), ("weighting", C.c_int32),
                ("batch", C.c_int32), ("scatter_mode", C.c_int32), ("d_l_out", C.c_void_p), ("d_tex_out", C.c_void_p),
                ("tex_dtype", C.c_int32), ("d_labels", C.c_void_p), ("d_images", C.c_void_p)]


_lib = None
_lock = threading.Lock()
_p, _i32, _i64 = C.c_void_p, C.c_int32, C.c_int64


def lib():
    """The loaded HIP library (raises if it was not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"semfuse HIP library missing: {LIB_PATH} (build it with "
                                   "`python -c 'import __graft_entry__ as g; g.build()'`)")
            L = C.CDLL(LIB_PATH)
            L.lf_last_error.restype = C.c_char_p
            L.lf_version.restype = C.c_char_p
            L.lf_mesh_sizes.argtypes = [C.POINTER(_MeshOpts), _i64, _i64, _p, C.POINTER(_i64), C.POINTER(_i64)]
            L.lf_load_mesh.argtypes = [C.POINTER(_MeshOpts), _p, _i64, _p, _i64, _p, _p, _i64, _p, _p, _i64, _p,
                                       C.POINTER(_p)]
            L.lf_reset.argtypes = [_p, _p]
            L.lf_frame_ws_bytes.argtypes = [_p, _i32, _i32, _i32, _i32, _i32, C.POINTER(_i64)]
            L.lf_fuse_frames.argtypes = [_p, _p, _i32, _i32, _i32, _p, _i32, _p, _p, _p, _i32, _p, _p, _i64, _i32,
                                         _i32, _p]
            L.lf_fuse_frames_noalloc.argtypes = [_p, _p, _i32, _i32, _i32, _p, _i32, _p, _p, _p, _i32, _p, _i32,
                                                 _i32, _p]
            L.lf_set_window.argtypes = [_p, _i64, _i64, _p, _p]
            L.lf_label_agreement.argtypes = [_p, _i32, _p, _p, _p, _i32, _i32, _i32, _i32, _p, _p, _p]
            L.lf_finalize.argtypes = [_p, _p, _i32, _p, _p]
            L.lf_render_labels.argtypes = [_p, _p, _i32, _i32, _i32, _p, _p, _p, _p, _p, _i64, _p]
            L.lf_rasterize.argtypes = [_p, _p, _i32, _i32, _i32, _p, _p, _p, _p, _i64, _p]
            L.lf_free_mesh.argtypes = [_p]
            L.lf_free_mesh.restype = None
            L.lf_profile_enable.argtypes = [_p, _i32]
            L.lf_profile_read.argtypes = [_p, _p]
            L.lf_mlp_sizes.argtypes = [C.POINTER(_i32), C.POINTER(_i64)]
            L.lf_mlp_pack.argtypes = [_p, _p, _p]
            L.lf_mlp_bind.argtypes = [_p, _p]
            L.lf_mlp_forward.argtypes = [_p, _p, _i64, _p, _p]
            L.lf_mlp_grad.argtypes = [_p, _p, _p, _i64, _p, _p, _p]
            L.lf_adam_step.argtypes = [_p, _p, _p, _p, _i64, C.c_float, C.c_float, C.c_float, C.c_float, _i32, _p]
            L.lf_extract_features.argtypes = [_p, _p, _i32, _i32, _i32, _p, _i32, _p, _p, _p, _p, _p, _p, _p, _i64,
                                              _p, _p, _i64, _p]
            L.lf_fuse_ws_bytes.argtypes = [_p, _i32, _i32, _i32, _i32, _i32, _i32, _p, C.POINTER(_i64)]
            L.lf_area_ws_bytes.argtypes = [_p, _i32, _i32, _i32, C.POINTER(_i64)]
            L.lf_set_weight_mix.argtypes = [_p, C.c_float]
            L.lf_triangle_max_pixels.argtypes = [_p, _p, _i32, _i32, _i32, _p, _p, _i64, _p]
            L.lf_texel_resolution.argtypes = [_p, _i64, C.c_float, _p, _p]
            L.lf_set_tuning.argtypes = [_p, C.POINTER(_Tuning)]
            L.lf_get_tuning.argtypes = [_p, C.POINTER(_Tuning)]
            L.lf_set_overlap.argtypes = [_p, _i32]
            L.lf_batch_ws_bytes.argtypes = [C.POINTER(_SceneJob), _i32, C.POINTER(_i64)]
            L.lf_fuse_batch.argtypes = [C.POINTER(_SceneJob), _i32, _p, _i64, _p]
            L.lf_graph_capture_batch.argtypes = [C.POINTER(_SceneJob), _i32, _p, _i64, _p, C.POINTER(_p)]
            L.lf_graph_launch.argtypes = [_p, _p]
            L.lf_graph_free.argtypes = [_p]
            L.lf_graph_free.restype = None
            for name in ("lf_mesh_sizes", "lf_load_mesh", "lf_reset", "lf_frame_ws_bytes", "lf_fuse_frames",
                         "lf_finalize", "lf_render_labels", "lf_rasterize", "lf_profile_enable", "lf_profile_read",
                         "lf_mlp_sizes", "lf_mlp_pack", "lf_mlp_bind", "lf_mlp_forward", "lf_mlp_grad",
                         "lf_adam_step", "lf_extract_features", "lf_set_tuning", "lf_get_tuning",
                         "lf_batch_ws_bytes", "lf_fuse_batch", "lf_graph_capture_batch", "lf_graph_launch",
                         "lf_fuse_ws_bytes", "lf_area_ws_bytes", "lf_triangle_max_pixels", "lf_texel_resolution",
                         "lf_set_weight_mix", "lf_set_overlap", "lf_set_window",
                         "lf_label_agreement", "lf_fuse_frames_noalloc"):
                getattr(L, name).restype = _i32
            _lib = L
    return _lib


def _check(st):
    if st != LF_OK:
        raise SemfuseError(st, lib().lf_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda(t, name, dtype=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def _probs_arg(probs, scale):
    """(dtype enum, strides array, scale) of a probability tensor [F, c, H, W]."""
    _need_cuda(probs, "probs")
    if probs.dtype == torch.float32:
        dt = F32
    elif probs.dtype == torch.uint8:
        dt = FP8_E4M3
        _need_cuda(scale, "scale", torch.float32)
        scale = scale.contiguous()
    else:
        raise TypeError("probs must be float32 or uint8 E4M3 codes")
    return dt, (C.c_int64 * 4)(*probs.stride()), scale


def version() -> str:
    return lib().lf_version().decode()


def mesh_sizes(n_vertices, n_faces, s=1, scheme=SPLIT, n_classes=40, aggregator=AGG_SUM, s_face=None,
               z_near=0.05):
    """(n_texels, mesh workspace bytes) -- lf_mesh_sizes."""
    o = _MeshOpts(scheme, s, n_classes, aggregator, F32, z_near)
    nx, ws = _i64(), _i64()
    hs = None
    if s_face is not None:
        import numpy as np
        arr = np.ascontiguousarray(s_face, dtype=np.int32)
        hs = arr.ctypes.data_as(_p)
    _check(lib().lf_mesh_sizes(C.byref(o), int(n_vertices), int(n_faces), hs, C.byref(nx), C.byref(ws)))
    return nx.value, ws.value


class Mesh:
    """A loaded mesh with its caller-owned accumulator (lf_load_mesh)."""

    def __init__(self, vertices: torch.Tensor, faces: torch.Tensor, *, n_classes: int, s: int = 1,
                 scheme: int = SPLIT, aggregator: int = AGG_SUM, s_face: torch.Tensor | None = None,
                 z_near: float = 0.05, keep_weights: bool = True, accum_dtype=torch.float32,
                 whole_texture: bool = True):
        _need_cuda(vertices, "vertices", torch.float32)
        _need_cuda(faces, "faces", torch.int32)
        vertices = vertices.contiguous()
        faces = faces.contiguous()
        self.device = vertices.device
        self.c = int(n_classes)
        self.opts = _MeshOpts(scheme, s, n_classes, aggregator, _TEX_DT[accum_dtype], z_near)
        hs = None if s_face is None else s_face.detach().cpu().to(torch.int32).numpy()
        self.n_texels, ws_bytes = mesh_sizes(vertices.shape[0], faces.shape[0], s, scheme, n_classes, aggregator,
                                             hs, z_near)
        self.vertices = vertices
        self.n_faces = int(faces.shape[0])
        self.ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=self.device)
        # whole_texture=False: no accumulator of all rows (the texture is fused
        # window by window, see set_window / fuse_windowed)
        self.accum = torch.empty((self.n_texels, self.c), dtype=accum_dtype, device=self.device) \
            if whole_texture else None
        self.wsum = torch.empty(self.n_texels, dtype=torch.float32, device=self.device) \
            if (whole_texture and (keep_weights or aggregator == AGG_MUL)) else None
        self.accum_dtype = accum_dtype
        self.aggregator = aggregator
        self.win = (0, self.n_texels if whole_texture else 0)
        sf = None
        if s_face is not None:
            sf = s_face.to(device=self.device, dtype=torch.int32).contiguous()
        h = _p()
        _check(lib().lf_load_mesh(C.byref(self.opts), _ptr(vertices), vertices.shape[0], _ptr(faces), faces.shape[0],
                                  _ptr(sf), _ptr(self.ws), self.ws.numel(), _ptr(self.accum), _ptr(self.wsum),
                                  self.n_texels, _stream(), C.byref(h)))
        self._h = h
        self._fws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lf_free_mesh(h)
            self._h = None

    # -- workspace -----------------------------------------------------------------
    def frame_ws(self, H, W, batch, weighting=W_PIXEL, scatter_mode=SCATTER_AUTO, probs=None):
        """Workspace tensor for frames of H x W processed ``batch`` at a time
        (exact for ``probs``' dtype and layout when given)."""
        n = _i64()
        if probs is not None:
            dt = F32 if probs.dtype == torch.float32 else FP8_E4M3
            strides = (C.c_int64 * 4)(*probs.stride())
            _check(lib().lf_fuse_ws_bytes(self._h, H, W, batch, weighting, scatter_mode, dt, strides, C.byref(n)))
            key = (H, W, batch, weighting, scatter_mode, dt, tuple(probs.stride()))
        else:
            _check(lib().lf_frame_ws_bytes(self._h, H, W, batch, weighting, scatter_mode, C.byref(n)))
            key = (H, W, batch, weighting, scatter_mode)
        t = self._fws.get(key)
        if t is None or t.numel() < n.value:
            self._fws.clear()
            t = torch.empty(n.value, dtype=torch.uint8, device=self.device)
            self._fws[key] = t
        return t

    # -- C-ABI calls -----------------------------------------------------------------
    def reset(self):
        _check(lib().lf_reset(self._h, _stream()))

    def _fuse_args(self, cams, probs, scale, valid, l_out, batch):
        F, c, H, W = probs.shape
        if c != self.c:
            raise ValueError(f"probs has {c} classes, mesh has {self.c}")
        _need_cuda(cams, "cams", torch.float32)
        _need_cuda(probs, "probs")
        _need_cuda(valid, "valid", torch.uint8)
        _need_cuda(l_out, "l_out", torch.int32)
        cams = cams.contiguous()
        if cams.shape != (F, 16):
            raise ValueError("cams must be [F, 16]")
        dt, strides, scale = _probs_arg(probs, scale)
        if valid is not None:
            valid = valid.contiguous()
        if l_out is not None and (not l_out.is_contiguous() or tuple(l_out.shape) != (F, H, W)):
            raise ValueError("l_out must be a contiguous [F, H, W] int32 tensor")
        b = max(1, min(int(batch), F))
        return F, H, W, cams, dt, strides, scale, valid, b

    def fuse_frames(self, cams: torch.Tensor, probs: torch.Tensor, *, scale=None, valid=None,
                    weighting=W_PIXEL, l_out=None, batch=16, scatter_mode=SCATTER_AUTO, ws=None):
        """lf_fuse_frames: probs is [F, c, H, W] (any strides) float32, or uint8
        E4M3 codes with ``scale`` [F, H, W]."""
        F, H, W, cams, dt, strides, scale, valid, b = self._fuse_args(cams, probs, scale, valid, l_out, batch)
        if ws is None:
            ws = self.frame_ws(H, W, b, weighting, scatter_mode, probs=probs)
        _check(lib().lf_fuse_frames(self._h, _ptr(cams), F, H, W, _ptr(probs), dt, strides, _ptr(scale), _ptr(valid),
                                    weighting, _ptr(l_out), _ptr(ws), ws.numel(), b, scatter_mode, _stream()))

    def fuse_frames_noalloc(self, cams: torch.Tensor, probs: torch.Tensor, *, scale=None, valid=None,
                            weighting=W_PIXEL, l_out=None, batch=16, scatter_mode=SCATTER_AUTO):
        """lf_fuse_frames_noalloc: lf_fuse_frames with the library's static
        per-device scratch (NOALLOC_SCRATCH_BYTES) as the frame workspace."""
        F, H, W, cams, dt, strides, scale, valid, b = self._fuse_args(cams, probs, scale, valid, l_out, batch)
        with torch.cuda.device(self.device):
            _check(lib().lf_fuse_frames_noalloc(self._h, _ptr(cams), F, H, W, _ptr(probs), dt, strides, _ptr(scale),
                                                _ptr(valid), weighting, _ptr(l_out), b, scatter_mode, _stream()))

    def finalize(self, tex_dtype=torch.float32, want_tex=True):
        """lf_finalize -> (texture [rows, c] or None, labels [rows] uint8) of the
        current texel-row window (all n_texels rows unless a window is set)."""
        n = self.win[1]
        tex = torch.empty((n, self.c), dtype=tex_dtype, device=self.device) if want_tex else None
        lab = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().lf_finalize(self._h, _ptr(tex), _TEX_DT[tex_dtype], _ptr(lab), _stream()))
        return tex, lab

    def render_labels(self, labels, *, l=None, cams=None, H=None, W=None, valid=None, out=None, batch=8):
        """lf_render_labels from stored rows ``l`` [F,H,W], or by re-rendering ``cams``."""
        if l is not None:
            F, H, W = l.shape
            _need_cuda(l, "l", torch.int32)
            l = l.contiguous()
        else:
            F = cams.shape[0]
        _need_cuda(labels, "labels", torch.uint8)
        _need_cuda(valid, "valid", torch.uint8)
        if valid is not None:
            valid = valid.contiguous()
        if out is None:
            out = torch.empty((F, H, W), dtype=torch.uint8, device=self.device)
        ws = None
        if l is None:
            _need_cuda(cams, "cams", torch.float32)
            cams = cams.contiguous()
            ws = self.frame_ws(H, W, max(1, min(batch, F)))
        _check(lib().lf_render_labels(self._h, _ptr(cams), F, H, W, _ptr(l), _ptr(valid), _ptr(labels), _ptr(out),
                                      _ptr(ws), 0 if ws is None else ws.numel(), _stream()))
        return out

    def rasterize(self, cams, H, W, batch=8, want=("tri", "l", "z")):
        """lf_rasterize -> dict of [F, H, W] tensors (tri int32, l int32, z float32)."""
        _need_cuda(cams, "cams", torch.float32)
        cams = cams.contiguous()
        F = cams.shape[0]
        out = {}
        for k, dt in (("tri", torch.int32), ("l", torch.int32), ("z", torch.float32)):
            out[k] = torch.empty((F, H, W), dtype=dt, device=self.device) if k in want else None
        ws = self.frame_ws(H, W, max(1, min(batch, F)))
        _check(lib().lf_rasterize(self._h, _ptr(cams), F, H, W, _ptr(out["tri"]), _ptr(out["l"]), _ptr(out["z"]),
                                  _ptr(ws), ws.numel(), _stream()))
        return out

    def set_window(self, row_lo=0, n_rows=None, accum=None, wsum=None):
        """lf_set_window: accumulate only texel rows [row_lo, row_lo + n_rows)
        into ``accum`` [n_rows, c] (and ``wsum`` [n_rows]); no arguments restore
        the whole-texture accumulator given at load."""
        n_rows = self.n_texels if n_rows is None else int(n_rows)
        _need_cuda(accum, "accum", self.accum_dtype)
        _need_cuda(wsum, "wsum", torch.float32)
        if accum is not None and (not accum.is_contiguous() or tuple(accum.shape) != (n_rows, self.c)):
            raise ValueError("accum must be a contiguous [n_rows, c] tensor")
        _check(lib().lf_set_window(self._h, int(row_lo), n_rows, _ptr(accum), _ptr(wsum)))
        self.win = (int(row_lo), n_rows)
        self._win_bufs = (accum, wsum)
        self._fws.clear()

    def fuse_windowed(self, cams, probs, *, window_rows, scale=None, valid=None, weighting=W_PIXEL, batch=16,
                      scatter_mode=SCATTER_AUTO, tex_dtype=torch.float32, labels=None, tex_out=None):
        """Out-of-core fusion: the texture is fused ``window_rows`` texel rows
        at a time (every window renders all frames again and aggregates only
        its rows into a device buffer of window_rows x c), normalised, and its
        rows copied out.  Returns (texture [n_texels, c] in ``tex_out`` -- by
        default pinned host memory -- and labels [n_texels] uint8 on the
        device, for render_labels).  The whole-texture state is restored
        afterwards."""
        window_rows = max(1, min(int(window_rows), self.n_texels))
        if labels is None:
            labels = torch.empty(self.n_texels, dtype=torch.uint8, device=self.device)
        if tex_out is None:
            tex_out = torch.empty((self.n_texels, self.c), dtype=tex_dtype, pin_memory=True)
        acc = torch.empty((window_rows, self.c), dtype=self.accum_dtype, device=self.device)
        ws = torch.empty(window_rows, dtype=torch.float32, device=self.device) if self.aggregator == AGG_MUL else None
        saved = self.win
        for lo in range(0, self.n_texels, window_rows):
            n = min(window_rows, self.n_texels - lo)
            self.set_window(lo, n, acc[:n], None if ws is None else ws[:n])
            self.reset()
            self.fuse_frames(cams, probs, scale=scale, valid=valid, weighting=weighting, batch=batch,
                             scatter_mode=scatter_mode)
            t, lab = self.finalize(tex_dtype)
            labels[lo:lo + n].copy_(lab)
            tex_out[lo:lo + n].copy_(t, non_blocking=tex_out.is_pinned())
        torch.cuda.current_stream().synchronize()
        if saved[1] == self.n_texels and self.accum is not None:
            self.set_window()
        else:
            self.set_window(0, 0, acc[:0], None if ws is None else ws[:0])
        return tex_out, labels

    def set_weight_mix(self, alpha: float):
        """lf_set_weight_mix: alpha of weighting=W_MIX ((1 - alpha) w^(P) + alpha w^(I))."""
        _check(lib().lf_set_weight_mix(self._h, float(alpha)))

    # -- texel resolution from the worst-case frame ---------------------------------------
    def triangle_max_pixels(self, cams, H, W, area=None, batch=16):
        """lf_triangle_max_pixels -> int32 [T]: most pixels each triangle covers in any frame
        (accumulates into ``area`` when given)."""
        _need_cuda(cams, "cams", torch.float32)
        cams = cams.contiguous()
        if area is None:
            area = torch.zeros(self.n_faces, dtype=torch.int32, device=self.device)
        _need_cuda(area, "area", torch.int32)
        b = max(1, min(int(batch), cams.shape[0]))
        n = _i64()
        _check(lib().lf_area_ws_bytes(self._h, H, W, b, C.byref(n)))
        ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        _check(lib().lf_triangle_max_pixels(self._h, _ptr(cams), cams.shape[0], H, W, _ptr(area), _ptr(ws), ws.numel(),
                                            _stream()))
        return area

    # -- tuning and jobs ----------------------------------------------------------------
    def set_tuning(self, tile=32, gather_unroll=8, small_px=48, gather_waves=8, learned_in_gather=0):
        """lf_set_tuning (results do not depend on it)."""
        _check(lib().lf_set_tuning(self._h, C.byref(_Tuning(tile, gather_unroll, small_px, gather_waves,
                                                            1 if learned_in_gather else 0))))
        self._fws.clear()

    def set_overlap(self, enabled=True):
        """lf_set_overlap: gathers on the mesh's second stream (True) or on the
        caller's stream (False); results do not depend on it."""
        _check(lib().lf_set_overlap(self._h, 1 if enabled else 0))

    def get_tuning(self):
        t = _Tuning()
        _check(lib().lf_get_tuning(self._h, C.byref(t)))
        return {"tile": t.tile, "gather_unroll": t.gather_unroll, "small_px": t.small_px,
                "gather_waves": t.gather_waves, "learned_in_gather": t.learned_in_gather}

    def job(self, cams, probs, *, scale=None, valid=None, pool=0, weighting=W_PIXEL, batch=16,
            scatter_mode=SCATTER_AUTO, l_out=None, tex_dtype=None, images=False):
        """A complete fusion of this mesh for fuse_batch / Graph: returns a
        SceneJob whose outputs (``labels``, ``tex``, ``images``, ``l``) are
        allocated here.  With ``pool`` > 0, ``probs`` / ``scale`` / ``valid``
        hold ``pool`` input frames and frame f reads input frame f % pool."""
        F = cams.shape[0]
        Fi, c, H, W = probs.shape
        if c != self.c:
            raise ValueError(f"probs has {c} classes, mesh has {self.c}")
        if pool == 0 and Fi != F:
            raise ValueError("without a pool, probs needs one frame per camera")
        if pool > 0 and Fi < pool:
            raise ValueError("probs holds fewer frames than the pool")
        _need_cuda(cams, "cams", torch.float32)
        _need_cuda(valid, "valid", torch.uint8)
        cams = cams.contiguous()
        dt, strides, scale = _probs_arg(probs, scale)
        if valid is not None:
            valid = valid.contiguous()
        if images and l_out is None:
            l_out = torch.empty((F, H, W), dtype=torch.int32, device=self.device)
        tex = torch.empty((self.n_texels, self.c), dtype=tex_dtype, device=self.device) if tex_dtype else None
        labels = torch.empty(self.n_texels, dtype=torch.uint8, device=self.device)
        imgs = torch.empty((F, H, W), dtype=torch.uint8, device=self.device) if images else None
        st = _SceneJob(self._h.value, cams.data_ptr(), F, H, W, probs.data_ptr(), dt, strides,
                       None if scale is None else scale.data_ptr(), None if valid is None else valid.data_ptr(),
                       int(pool), int(weighting), int(batch), int(scatter_mode),
                       None if l_out is None else l_out.data_ptr(), None if tex is None else tex.data_ptr(),
                       _TEX_DT[tex_dtype] if tex_dtype else F32, labels.data_ptr(),
                       None if imgs is None else imgs.data_ptr())
        return SceneJob(self, st, (cams, probs, scale, valid), l_out, tex, labels, imgs)

    # -- learned weighting ------------------------------------------------------------
    def bind_mlp(self, mlp):
        """lf_mlp_bind: fuse with ``weighting=W_LEARNED`` using ``mlp`` (a WeightMLP
        or a packed uint8 tensor; None unbinds).  The mesh keeps a reference."""
        packed = None if mlp is None else (mlp.packed if hasattr(mlp, "packed") else mlp)
        _check(lib().lf_mlp_bind(self._h, _ptr(packed)))
        self._mlp = packed

    def extract_features(self, cams, probs, *, scale=None, valid=None, labels=None, cap=None, want_pix=True,
                         batch=8):
        """lf_extract_features -> (phi [n, 8], target [n] or None, pix [n] or None);
        observations come in unspecified order."""
        F, c, H, W = probs.shape
        if c != self.c:
            raise ValueError(f"probs has {c} classes, mesh has {self.c}")
        _need_cuda(cams, "cams", torch.float32)
        _need_cuda(valid, "valid", torch.uint8)
        _need_cuda(labels, "labels", torch.uint8)
        cams = cams.contiguous()
        dt, strides, scale = _probs_arg(probs, scale)
        if valid is not None:
            valid = valid.contiguous()
        cap = F * H * W if cap is None else int(cap)
        phi = torch.empty((max(cap, 1), 8), dtype=torch.float32, device=self.device)
        tgt = torch.empty(max(cap, 1), dtype=torch.float32, device=self.device) if labels is not None else None
        pix = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device) if want_pix else None
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        ws = self.frame_ws(H, W, max(1, min(batch, F)), W_LEARNED, SCATTER_ATOMIC)
        _check(lib().lf_extract_features(self._h, _ptr(cams), F, H, W, _ptr(probs), dt, strides, _ptr(scale),
                                         _ptr(valid), _ptr(labels), _ptr(phi), _ptr(tgt), _ptr(pix), cap, _ptr(count),
                                         _ptr(ws), ws.numel(), _stream()))
        n = min(int(count.item()), cap)
        return phi[:n], (tgt[:n] if tgt is not None else None), (pix[:n] if pix is not None else None)


def mlp_sizes():
    """(number of binary32 master parameters, bytes of the packed form)."""
    n, b = _i32(), _i64()
    _check(lib().lf_mlp_sizes(C.byref(n), C.byref(b)))
    return n.value, b.value


class WeightMLP:
    """Parameters of the learned weight network on one device: binary32 master
    copy, Adam moments and the packed bfloat16 form the kernels read."""

    def __init__(self, device="cuda", params: torch.Tensor | None = None, seed: int = 0):
        n, nb = mlp_sizes()
        self.n_params = n
        self.device = torch.device(device)
        if params is None:
            params = init_params(seed)
        params = torch.as_tensor(params, dtype=torch.float32)
        if params.numel() != n:
            raise ValueError(f"expected {n} parameters, got {params.numel()}")
        self.params = params.reshape(-1).to(self.device).contiguous()
        self.m = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=self.device)
        self.grad_buf = torch.empty(n, dtype=torch.float32, device=self.device)
        self.loss_buf = torch.empty(1, dtype=torch.float32, device=self.device)
        self.packed = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.t = 0
        self.pack()

    def pack(self):
        _check(lib().lf_mlp_pack(_ptr(self.params), _ptr(self.packed), _stream()))

    def forward(self, phi: torch.Tensor) -> torch.Tensor:
        _need_cuda(phi, "phi", torch.float32)
        phi = phi.contiguous()
        w = torch.empty(phi.shape[0], dtype=torch.float32, device=self.device)
        _check(lib().lf_mlp_forward(_ptr(self.packed), _ptr(phi), phi.shape[0], _ptr(w), _stream()))
        return w

    def loss_grad(self, phi: torch.Tensor, target: torch.Tensor):
        """(loss [1] tensor, gradient [n_params] tensor) -- views of internal buffers."""
        _need_cuda(phi, "phi", torch.float32)
        _need_cuda(target, "target", torch.float32)
        phi, target = phi.contiguous(), target.contiguous()
        _check(lib().lf_mlp_grad(_ptr(self.packed), _ptr(phi), _ptr(target), phi.shape[0], _ptr(self.grad_buf),
                                 _ptr(self.loss_buf), _stream()))
        return self.loss_buf, self.grad_buf

    def adam(self, grad: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on the master parameters, then repack."""
        self.t += 1
        _check(lib().lf_adam_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(grad), self.n_params, lr, beta1,
                                  beta2, eps, self.t, _stream()))
        self.pack()


def init_params(seed: int = 0) -> torch.Tensor:
    """He-normal weights, zero biases (host float32 [n_params])."""
    n, _ = mlp_sizes()
    g = torch.Generator().manual_seed(int(seed))
    NI, NH = 8, 64
    p = torch.zeros(n, dtype=torch.float32)
    o = 0
    p[o:o + NH * NI] = torch.randn(NH * NI, generator=g) * (2.0 / NI) ** 0.5
    o += NH * NI + NH
    p[o:o + NH * NH] = torch.randn(NH * NH, generator=g) * (2.0 / NH) ** 0.5
    o += NH * NH + NH
    p[o:o + NH] = torch.randn(NH, generator=g) * (1.0 / NH) ** 0.5
    return p


class SceneJob:
    """One scene's complete fusion (an lf_scene_job) with the tensors it uses."""

    def __init__(self, mesh, st, inputs, l, tex, labels, images):
        self.mesh, self.st, self.inputs = mesh, st, inputs
        self.l, self.tex, self.labels, self.images = l, tex, labels, images


def _job_array(jobs):
    arr = (_SceneJob * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        arr[i] = j.st
    return arr


def batch_ws(jobs, device="cuda"):
    """Workspace tensor sized by lf_batch_ws_bytes for these jobs."""
    n = _i64()
    _check(lib().lf_batch_ws_bytes(_job_array(jobs), len(jobs), C.byref(n)))
    return torch.empty(n.value, dtype=torch.uint8, device=device)


def fuse_batch(jobs, ws=None):
    """lf_fuse_batch on the current stream."""
    if ws is None:
        ws = batch_ws(jobs)
    _check(lib().lf_fuse_batch(_job_array(jobs), len(jobs), _ptr(ws), ws.numel(), _stream()))
    return ws


class Graph:
    """lf_graph_capture_batch / lf_graph_launch: the jobs' whole launch
    sequence as one executable HIP graph.  Captured on a private stream
    (default priority); the graph keeps the jobs and workspace alive."""

    def __init__(self, jobs, ws=None):
        self.jobs = list(jobs)
        self.ws = batch_ws(self.jobs) if ws is None else ws
        self.stream = torch.cuda.Stream()
        self.stream.wait_stream(torch.cuda.current_stream())
        h = _p()
        with torch.cuda.stream(self.stream):
            _check(lib().lf_graph_capture_batch(_job_array(self.jobs), len(self.jobs), _ptr(self.ws), self.ws.numel(),
                                                C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def launch(self):
        """Replay on the current stream."""
        _check(lib().lf_graph_launch(self._h, _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lf_graph_free(h)
            self._h = None


def label_agreement(probs, images, *, scale=None, valid=None, counts=None):
    """lf_label_agreement -> int64 [2] device tensor: (labelled valid pixels,
    those whose label is the pixel's own argmax), accumulated into ``counts``."""
    F, c, H, W = probs.shape
    dt, strides, scale = _probs_arg(probs, scale)
    _need_cuda(images, "images", torch.uint8)
    _need_cuda(valid, "valid", torch.uint8)
    images = images.contiguous()
    if valid is not None:
        valid = valid.contiguous()
    if counts is None:
        counts = torch.zeros(2, dtype=torch.int64, device=probs.device)
    _check(lib().lf_label_agreement(_ptr(probs), dt, strides, _ptr(scale), _ptr(valid), c, F, H, W, _ptr(images),
                                    _ptr(counts), _stream()))
    return counts


def texel_resolution(area: torch.Tensor, gamma: float) -> torch.Tensor:
    """lf_texel_resolution: per-face s = max(1, ceil(gamma * sqrt(area))) (int32 [T])."""
    _need_cuda(area, "area", torch.int32)
    area = area.contiguous()
    s = torch.empty_like(area)
    _check(lib().lf_texel_resolution(_ptr(area), area.numel(), float(gamma), _ptr(s), _stream()))
    return s
