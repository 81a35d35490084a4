"""Autotuner of the fusion's launch parameters.

For one (device, image size, class count, input dtype and layout, mesh size,
weighting) it times candidates of six knobs on the first frames of the
caller's own input (at least three batches of them, so that the overlap of
one batch's gather with the next batch's raster is part of the timing):
frames per batch (8 to 128), scatter mode (texel-sorted when a pixel's
classes are contiguous, staged texel-sorted for planar FP32 inputs, LDS-hash
atomic always), raster tile edge (16, 32), the largest triangle box
rasterized by one lane (12, 24, 48, 96 pixels), the sorted gather's unroll
(4, 8) and the resident waves per CU its grid is sized for (8, 16, 32).  The
search is coordinate descent from the library defaults: each knob in turn is
swept with the others held, and a value replaces the current one only when
it is more than 1% faster (smaller differences are timing noise).  The choice is
cached in a JSON file keyed by that tuple.  Results never depend on the
choice; only speed does.  Timing uses events on the stream the library
launches on; the mesh's accumulator is cleared afterwards.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import threading

import torch

from . import semfuse as sf

BATCHES = (8, 16, 32, 64, 128)
TILES = (16, 32)
SMALL = (12, 24, 48, 96)
UNROLLS = (4, 8)
GATHER_WAVES = (8, 16, 32)
MIN_GAIN = 0.01     # a candidate replaces the incumbent only when faster by more than this (timing noise)
_lock = threading.Lock()


def default_cache_path() -> str:
    return os.environ.get("SEMFUSE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "semfuse", "tune.json"))


def cache_key(mesh: sf.Mesh, H: int, W: int, probs: torch.Tensor, weighting: int) -> str:
    props = torch.cuda.get_device_properties(mesh.device)
    arch = getattr(props, "gcnArchName", props.name)
    layout = "cl" if probs.stride(1) == 1 else "planar"
    tris = int(mesh.n_faces)
    return (f"{arch}|{W}x{H}|c{mesh.c}|{str(probs.dtype)[6:]}|{layout}|T2^{round(math.log2(max(tris, 1)))}"
            f"|x{round(mesh.n_texels / max(tris, 1))}|w{weighting}|agg{mesh.opts.aggregator}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def scatter_modes(probs: torch.Tensor):
    c = probs.shape[1]
    modes = [sf.SCATTER_ATOMIC]
    if probs.stride(1) == 1:
        modes.insert(0, sf.SCATTER_SORTED)
    elif probs.dtype == torch.float32 and c % 4 == 0 and c <= 60:
        modes.insert(0, sf.SCATTER_STAGED)
    return modes


def coordinate_descent(trial, start, sweeps, min_gain=MIN_GAIN):
    """Sweep each (knob, values) in turn with the other knobs held; a value
    replaces the current one only when its time is more than `min_gain`
    (relative) below the best so far.  The gather's knobs are skipped while
    the atomic scatter is chosen.  Returns (best configuration, its time)."""
    best = dict(start)
    best_ms = trial(best)
    for knob, values in sweeps:
        if knob in ("gather_unroll", "gather_waves") and best.get("scatter_mode") == sf.SCATTER_ATOMIC:
            continue                            # these only affect the sorted gather
        for v in values:
            cand = dict(best, **{knob: v})
            ms = trial(cand)
            if ms < best_ms * (1.0 - min_gain):
                best, best_ms = cand, ms
    return best, best_ms


def _ws_bytes(mesh, H, W, batch, weighting, mode, probs):
    n = C.c_int64()
    dt = sf.F32 if probs.dtype == torch.float32 else sf.FP8_E4M3
    strides = (C.c_int64 * 4)(*probs.stride())
    sf._check(sf.lib().lf_fuse_ws_bytes(mesh._h, H, W, batch, weighting, mode, dt, strides, C.byref(n)))
    return n.value


def _apply(mesh, cfg):
    mesh.set_tuning(cfg["tile"], cfg["gather_unroll"], cfg["small_px"], cfg["gather_waves"],
                    cfg.get("learned_in_gather", 0))


def autotune(mesh: sf.Mesh, cams: torch.Tensor, probs: torch.Tensor, *, scale=None, valid=None,
             weighting=sf.W_PIXEL, probe_frames=64, cache_path=None, force=False, ws_budget=8 << 30,
             repeats=2, log=None):
    """Best {batch, scatter_mode, tile, small_px, gather_unroll, gather_waves, ms_per_frame}
    for this mesh and input; applies the tuning to ``mesh`` and returns it."""
    F, c, H, W = probs.shape
    path = cache_path or default_cache_path()
    key = cache_key(mesh, H, W, probs, weighting)
    with _lock:
        table = _load(path)
    if not force and key in table:
        best = table[key]
        _apply(mesh, best)
        if log:
            log(f"[tune] cache hit {key}: {best}")
        return dict(best, cached=True)
    nf = max(1, min(F, probe_frames))
    timings = {}

    def trial(cfg):
        k = tuple(sorted(cfg.items()))
        if k in timings:
            return timings[k]
        b = min(cfg["batch"], nf)
        n = min(F, max(nf, 3 * b))
        cams_p, probs_p = cams[:n], probs[:n]
        scale_p = None if scale is None else scale[:n]
        valid_p = None if valid is None else valid[:n]
        _apply(mesh, cfg)
        if _ws_bytes(mesh, H, W, b, weighting, cfg["scatter_mode"], probs_p) > ws_budget:
            timings[k] = math.inf
            return math.inf
        ws = mesh.frame_ws(H, W, b, weighting, cfg["scatter_mode"], probs=probs_p)

        def run():
            mesh.fuse_frames(cams_p, probs_p, scale=scale_p, valid=valid_p, weighting=weighting, batch=b,
                             scatter_mode=cfg["scatter_mode"], ws=ws)
        run()                                   # warm-up (first touch of the workspace, code load)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(repeats):
            run()
        ev1.record()
        ev1.synchronize()
        timings[k] = ev0.elapsed_time(ev1) / (repeats * n)
        return timings[k]

    modes = scatter_modes(probs)
    batches = [b for b in BATCHES if b <= max(nf, BATCHES[0])]
    start = {"batch": min(32, batches[-1]), "scatter_mode": modes[0], "tile": 32, "small_px": 48,
             "gather_unroll": 8, "gather_waves": 8}
    sweeps = [("batch", batches), ("scatter_mode", modes), ("tile", TILES), ("small_px", SMALL),
              ("gather_unroll", UNROLLS), ("gather_waves", GATHER_WAVES)]
    if weighting == sf.W_LEARNED:
        # where the network runs: inside the gather, or a separate pass first
        start["learned_in_gather"] = 0
        sweeps.append(("learned_in_gather", (0, 1)))
    best, best_ms = coordinate_descent(trial, start, sweeps)
    mesh.reset()
    mesh._fws.clear()
    if not math.isfinite(best_ms):
        raise RuntimeError("no tuning candidate fits the workspace budget")
    choice = dict(best, ms_per_frame=best_ms, probe_frames=nf, n_candidates=len(timings))
    _apply(mesh, choice)
    with _lock:
        table = _load(path)
        table[key] = choice
        _store(path, table)
    if log:
        log(f"[tune] {key}: {len(timings)} candidates, best {choice}")
    return dict(choice, cached=False)
