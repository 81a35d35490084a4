#!/usr/bin/env python3
"""Benchmark of the label-fusion hot path on one MI355X.

Workload (default): a procedural room of 501,908 triangles, SPLIT s = 3
(4,517,172 texels), 300 frames of 640x480 along a smooth random walk, c = 40,
FP32 probabilities resident in HBM in channels-last layout, 15 % wrong-class
blobs, 5 % pixels without depth.  One step = clear the accumulator, fuse all
300 frames (render to triangle/texel ids, sort by texel, gather-accumulate),
normalise + argmax every texel, render the labels back into all 300 frames.

Prints one JSON line: fused pixels/s, the dominant kernel's fraction of the
HBM roofline (algorithmic bytes / its HIP-event-timed launch duration), the
CPU oracle's rate on a bounded sample, the other input forms' throughput
(NCHW, FP8, w^(I), learned weight) and the label accuracy of the plain,
reduced-precision and learned forms on held-out small scenes.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused pixels/sec (c=40, 640×480) + % HBM roofline; learned/BF16 vs plain at label acc"
HBM_PEAK_GBS = 8000.0
STAGES = ["raster", "resolve", "scatter", "counts", "finalize", "render", "reset", "mlp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bucket_gather16_room500k_640x480_c40.txt")
ISO_GATHER_WAVES = 512      # gather grid when it has the device alone: 8x more groups than fit, rows balance


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Prof(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8)]


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("sorted.hip", "internal.h", "accum.h"):
        with open(os.path.join(ROOT, "paper_2111_11103_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


GATHER_KNOBS = ("batch", "scatter_mode", "gather_unroll", "gather_waves")   # what the gather's launch depends on


def measured_traffic(launch):
    """HBM bytes per fused pixel of the gather from the committed counter
    summary (one record per measured launch configuration), or None when the
    kernel's sources differ from those measured or no record has this
    launch's gather configuration."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.loads(fh.readline())       # first line: the figures; the rest: how they were taken
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != kernel_source_digest():
        return None
    for rec in t.get("records", []):
        if all(rec.get(k) == launch.get(k) for k in GATHER_KNOBS):
            return rec.get("bytes_per_px")
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_fuse_timed(work, n_frames: int, threads: int):
    """The CPU oracle (raster on `threads` host threads, binary64 fusion) on
    the first ``n_frames`` frames of the workload: (seconds, rows, A)."""
    import oracle
    sc = work.scene
    probs = work.probs[:n_frames].cpu().numpy()
    valid = work.valid[:n_frames].cpu().numpy()
    t0 = time.perf_counter()
    om = oracle.Mesh(sc.vertices, sc.faces, s=work.s, scheme=work.scheme)
    _, l = om.raster_frames(work.cams[:n_frames], work.H, work.W, threads=threads)
    A, _ = oracle.fuse(om.n_texels, sc.n_classes, l, probs, valid)
    return time.perf_counter() - t0, l, A


def cpu_baseline(work, n_frames: int, n_frames_1t: int):
    """The CPU oracle on the first ``n_frames`` frames with the box's threads
    (up to 16, its CPU share) and on the first ``n_frames_1t`` frames with one
    thread; fused pixels/s.  Also returns the oracle's rows and binary64
    texture of the larger sample, for the benchmark's own result check."""
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(threads, 16))
    px = work.H * work.W
    dt, l, A = oracle_fuse_timed(work, n_frames, threads)
    dt1, _, _ = oracle_fuse_timed(work, n_frames_1t, 1)
    res = {"value": n_frames * px / dt, "unit": "fused pixels/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n_frames} of {len(work.cams)} frames of the same workload (raster on {threads} "
                     f"threads, binary64 fusion on 1 thread), {dt:.1f} s",
           "one_thread": {"value": n_frames_1t * px / dt1, "cores": 1,
                          "sample": f"first {n_frames_1t} frames, raster and fusion on 1 thread, {dt1:.1f} s"},
           "cpu_model": cpu_model()}
    return res, l, A


def device_probe(dev, copy_mib=2048, n_atomics=1 << 26):
    """Measured ceilings of the device: a plain device-to-device copy (bytes
    read + written per second) and FP32 atomic additions per second (torch's
    index_add_) to scattered distinct addresses, to consecutive addresses
    (16 lanes per 64-byte line) and to 64 contended addresses."""
    import torch
    n = copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    copy_gbs = 5 * 2 * n * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    g = torch.Generator(device=dev).manual_seed(0)
    src = torch.ones(n_atomics, dtype=torch.float32, device=dev)
    out = torch.zeros(n_atomics, dtype=torch.float32, device=dev)
    cases = {"scattered_distinct": torch.randperm(n_atomics, device=dev, generator=g),
             "consecutive_distinct": torch.arange(n_atomics, device=dev),
             "contended_64_addresses": torch.arange(n_atomics, device=dev) % 64}
    rates = {}
    for name, idx in cases.items():
        out.index_add_(0, idx, src)
        e0.record()
        for _ in range(3):
            out.index_add_(0, idx, src)
        e1.record()
        e1.synchronize()
        rates[name] = 3 * n_atomics / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, out, cases
    torch.cuda.empty_cache()
    return {"copy_gbs": copy_gbs, "copy_bytes": 2 * n * 4,
            "fp32_atomic_add_g_per_s": rates, "atomic_ops_per_case": n_atomics}


def result_check(mesh, cams, probs, valid, l_oracle, A_oracle, batch, scatter, tol=1e-5):
    """The headline launch configuration run again on the oracle's sample of
    frames into a cleared accumulator: texel rows bit-exact, every fused
    entry within ``tol`` relative of the binary64 oracle."""
    import numpy as np
    import torch
    n = l_oracle.shape[0]
    l_g = torch.empty((n,) + tuple(l_oracle.shape[1:]), dtype=torch.int32, device=probs.device)
    mesh.reset()
    mesh.fuse_frames(cams[:n], probs[:n], valid=valid[:n], l_out=l_g, batch=batch, scatter_mode=scatter)
    torch.cuda.synchronize()
    rows_equal = bool(np.array_equal(l_g.cpu().numpy(), l_oracle))
    A_g = mesh.accum.cpu().numpy().astype(np.float64)
    err = np.abs(A_g - A_oracle)
    bad = int((err > tol * np.abs(A_oracle)).sum())
    worst = float((err / np.maximum(np.abs(A_oracle), 1e-300)).max())
    mesh.reset()
    return {"frames": n, "texel_rows_bit_exact": rows_equal, "entries": int(A_oracle.size),
            "entries_beyond_tol": bad, "tol_rel": tol, "max_rel_err": worst, "ok": rows_equal and bad == 0}


def accuracy_report(log_fn):
    """Pixel accuracy of the fusion forms on held-out small scenes (2,100
    triangles, c = 13, 20 frames 160x120, view-dependent noise, seeds
    200-209); the learned weight is first trained on seeds 100-149."""
    import numpy as np
    import torch
    from paper_2111_11103_amd import learned as LR
    from paper_2111_11103_amd import scenes as S
    from paper_2111_11103_amd import semfuse as sf
    t0 = time.time()
    phi, tgt = LR.training_set(range(100, 150), device="cuda", structured=True)
    mlp = sf.WeightMLP("cuda", seed=0)
    LR.train(mlp, phi, tgt, steps=1500, batch=32768, lr=2e-3)
    del phi, tgt
    acc = {k: [] for k in ("input", "pixel", "image", "learned", "bf16_texture", "fp16_texture", "fp8_input")}
    for sd in range(200, 210):
        w = S.config1(device="cuda", seed=sd, structured=True)
        r = LR.evaluate(w, mlp)
        for k in ("input", "pixel", "image", "learned"):
            acc[k].append(r[k])
        cams = torch.as_tensor(w.cams, dtype=torch.float32, device="cuda")
        l_rows = torch.empty((len(w.cams), w.H, w.W), dtype=torch.int32, device="cuda")
        seen = None
        for name, dt, fp8 in (("bf16_texture", torch.bfloat16, False), ("fp16_texture", torch.float16, False),
                              ("fp8_input", torch.float32, True)):
            mesh = LR.scene_mesh(w, "cuda")
            if fp8:
                q, scale = S.quantize_fp8(w.probs)
                mesh.fuse_frames(cams, q, scale=scale, valid=w.valid, l_out=l_rows)
            else:
                mesh.fuse_frames(cams, w.probs, valid=w.valid, l_out=l_rows)
            _, lab = mesh.finalize(dt)
            out = mesh.render_labels(lab, l=l_rows, valid=w.valid)
            seen = (l_rows >= 0) & (w.valid != 0)
            acc[name].append(float((out[seen].long() == w.gt[seen]).float().mean()))
    res = {k: float(np.mean(v)) for k, v in acc.items()}
    log_fn(f"[bench] accuracy report in {time.time() - t0:.1f} s: {res}")
    res["workload"] = ("held-out rooms (2,100 triangles, c=13, 20 frames 160x120, view-dependent noise, seeds "
                       "200-209); learned weight trained on seeds 100-149 by the library's kernels")
    return res, mlp


def weight_and_frame_sweeps(log_fn, seeds=range(200, 210)):
    """The evaluation's two sweeps on synthetic held-out rooms (2,100
    triangles, c = 13, 20 frames 160x120, view-dependent noise), with the
    evaluation's f_mul aggregator and triangles as texels (gamma = 0, s = 1):
    pixel accuracy for weights w = (1 - alpha) w^(P) + alpha w^(I) (Fig. 4a),
    and for frames taken at uniform intervals with w^(I) (Fig. 4b).  Fused
    labels are rendered into all 20 frames (pixels whose texel no fused frame
    saw render void and count as wrong)."""
    import numpy as np
    import torch
    from paper_2111_11103_amd import scenes as S
    from paper_2111_11103_amd import semfuse as sf
    alphas = (0.0, 0.25, 0.5, 0.75, 1.0)
    steps = (1, 2, 3, 4, 5, 10, 20)
    acc_a = {a: [] for a in alphas}
    acc_f = {st: [] for st in steps}
    for sd in seeds:
        w = S.config1(device="cuda", seed=sd, structured=True)
        sc = w.scene
        cams = torch.as_tensor(w.cams, dtype=torch.float32, device="cuda")
        seen = None

        def fused_accuracy(frames, weighting, alpha=None):
            nonlocal seen
            mesh = sf.Mesh(torch.as_tensor(sc.vertices, device="cuda"), torch.as_tensor(sc.faces, device="cuda"),
                           n_classes=sc.n_classes, s=1, scheme=sf.SPLIT, aggregator=sf.AGG_MUL)
            if alpha is not None:
                mesh.set_weight_mix(alpha)
            mesh.fuse_frames(cams[frames], w.probs[frames], valid=w.valid[frames], weighting=weighting)
            _, lab = mesh.finalize(want_tex=False)
            out = mesh.render_labels(lab, cams=cams, H=w.H, W=w.W, valid=w.valid)
            if seen is None:
                l = mesh.rasterize(cams, w.H, w.W, want=("l",))["l"]
                seen = (l >= 0) & (w.valid != 0)
            return float((out[seen].long() == w.gt[seen]).float().mean())

        for a in alphas:
            acc_a[a].append(fused_accuracy(slice(None), sf.W_MIX, a))
        for st in steps:
            acc_f[st].append(fused_accuracy(slice(None, None, st), sf.W_IMAGE))
    res = {"aggregator": "f_mul", "texels": "triangles (s = 1)",
           "accuracy_vs_alpha": {f"{a:g}": float(np.mean(v)) for a, v in acc_a.items()},
           "accuracy_vs_frame_fraction": {f"{1 / st:.3g}": float(np.mean(v)) for st, v in acc_f.items()},
           "workload": "held-out rooms (2,100 triangles, c=13, 20 frames 160x120, view-dependent noise, seeds "
                       "200-209); labels rendered into all 20 frames"}
    log_fn(f"[bench] weight / frame sweeps: {res}")
    return res


def learned_scale_report(mlp, log_fn, n_frames=1000, pool=16):
    """Learned weight at scale: a 2M-triangle room, SPLIT s = 4 (32M texels),
    1000 frames of 1296x968 (inputs cycled from a pool of 16), c = 40.
    Throughput of plain w^(P) vs the learned weight (network evaluated inside
    the gather, and in a separate pass first), and pixel accuracy of both on
    the pool's own 16 frames."""
    import torch
    from paper_2111_11103_amd import scenes as S
    from paper_2111_11103_amd import semfuse as sf
    t0 = time.time()
    sc = S.config2_scene(seed=0, target_tris=2_000_000)
    H, W = 968, 1296
    cams_np = S.random_walk_cameras(sc, n_frames, W, H, seed=0)
    probs, valid, gt = S.frame_inputs(sc, cams_np[:pool], H, W, margin=3.0, sigma=2.0, blob_frac=0.15,
                                      invalid_frac=0.05, seed=0, device="cuda")
    probs = probs.to(memory_format=torch.channels_last)
    dev = probs.device
    cams = torch.as_tensor(cams_np, device=dev)
    mesh = sf.Mesh(torch.as_tensor(sc.vertices, device=dev), torch.as_tensor(sc.faces, device=dev), n_classes=40,
                   s=4, scheme=sf.SPLIT, keep_weights=False)
    mesh.bind_mlp(mlp)
    log_fn(f"[bench] learned at scale: T={sc.n_faces} texels={mesh.n_texels} ready in {time.time() - t0:.0f} s")
    res = {"workload": f"room mesh {sc.n_faces} triangles, SPLIT s=4 ({mesh.n_texels} texels), {n_frames} frames "
                       f"{W}x{H} (input pool of {pool}), c=40"}
    tuning = mesh.get_tuning()
    for name, wt, site in (("plain", sf.W_PIXEL, 1), ("learned", sf.W_LEARNED, 1),
                           ("learned_separate_pass", sf.W_LEARNED, 0)):
        mesh.set_tuning(**dict(tuning, learned_in_gather=site))
        job = mesh.job(cams, probs, valid=valid, pool=pool, weighting=wt, batch=pool, scatter_mode=sf.SCATTER_SORTED)
        ws = sf.batch_ws([job])
        sf.fuse_batch([job], ws)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        sf.fuse_batch([job], ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - tt
        res[f"{name}_value"] = n_frames * H * W / dt
        res[f"{name}_ms"] = dt * 1e3
        if site == 1:
            # accuracy on the pool's own frames (their cameras, their ground truth)
            acc_job = mesh.job(cams[:pool], probs, valid=valid, weighting=wt, batch=pool, images=True)
            sf.fuse_batch([acc_job])
            torch.cuda.synchronize()
            seen = (acc_job.l >= 0) & (valid != 0)
            res[f"{name}_pixel_acc"] = float((acc_job.images[seen].long() == gt[seen]).float().mean())
            if "input_pixel_acc" not in res:
                res["input_pixel_acc"] = float((probs.argmax(1)[seen] == gt[seen]).float().mean())
            del acc_job
        del job, ws
        torch.cuda.empty_cache()
    mesh.set_tuning(**tuning)
    mesh.bind_mlp(None)
    log_fn(f"[bench] learned at scale: {res}")
    return res


def batched_report(log_fn, steps=2, scale=1.0):
    """Batched form: 16 rooms of uneven size (50k-2M triangles, SPLIT s = 1-4,
    100-1000 frames each at 640x480 or 1296x968, c = 40, cycled input pools),
    each scene's launch parameters chosen by the autotuner: the whole job
    (clear, fuse, normalise, render back, for every scene) as one
    lf_fuse_batch call (`value`), and captured as HIP graphs and replayed
    (`graph_value`)."""
    import torch
    from paper_2111_11103_amd import scenes as S
    from paper_2111_11103_amd import semfuse as sf
    from paper_2111_11103_amd import tune
    t0 = time.time()
    jobs, choices = [], []
    n_px = n_frames = n_tex = 0
    for i, p in enumerate(S.config4(device="cuda", scale=scale)):
        dev = p.probs.device
        mesh = sf.Mesh(torch.as_tensor(p.scene.vertices, device=dev), torch.as_tensor(p.scene.faces, device=dev),
                       n_classes=p.scene.n_classes, s=p.s, scheme=sf.SPLIT, keep_weights=False)
        probs = p.probs.to(memory_format=torch.channels_last)
        cams = torch.as_tensor(p.cams, device=dev)
        best = tune.autotune(mesh, cams[:p.pool], probs, valid=p.valid, probe_frames=p.pool)
        choices.append({k: best[k] for k in ("tile", "gather_unroll", "small_px", "gather_waves", "batch",
                                             "scatter_mode", "cached")})
        jobs.append(mesh.job(cams, probs, valid=p.valid, pool=p.pool, batch=best["batch"],
                             scatter_mode=best["scatter_mode"], images=True))
        F = len(p.cams)
        n_frames += F
        n_px += F * p.H * p.W
        n_tex += mesh.n_texels
        log_fn(f"[bench] batched scene {i}: T={p.scene.n_faces} s={p.s} texels={mesh.n_texels} {F} frames "
               f"{p.W}x{p.H} tuned {choices[-1]} ({time.time() - t0:.0f} s)")
    ws = sf.batch_ws(jobs)
    sf.fuse_batch(jobs, ws)                 # warm-up (first touch of the workspace)
    torch.cuda.synchronize()
    te = time.perf_counter()
    for _ in range(steps):
        sf.fuse_batch(jobs, ws)
    torch.cuda.synchronize()
    eager_s = (time.perf_counter() - te) / steps
    log_fn(f"[bench] batched call {eager_s * 1e3:.1f} ms ({n_px / eager_s / 1e9:.2f} G px/s)")
    g = sf.Graph(jobs, ws)
    g.launch()
    torch.cuda.synchronize()
    tg = time.perf_counter()
    for _ in range(steps):
        g.launch()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - tg) / steps
    log_fn(f"[bench] batched graph replay {graph_s * 1e3:.1f} ms ({n_px / graph_s / 1e9:.2f} G px/s)")
    return {"value": n_px / eager_s, "unit": "fused pixels/s", "ms_per_call": eager_s * 1e3, "calls": steps,
            "graph_value": n_px / graph_s, "ms_per_replay": graph_s * 1e3, "replays": steps,
            "scenes": len(jobs), "frames": n_frames, "pixels": n_px,
            "texels": n_tex, "workspace_bytes": ws.numel(), "tuning": choices,
            "workload": "16 rooms (seed 1000+i, T=50k*40^(i/15), SPLIT s=1+i%4, 100+60i frames, 640x480 even i / "
                        "1296x968 odd i, c=40, input pools of 16 / 8 frames), one lf_fuse_batch call"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--batch", type=int, default=0, help="frames per batch; 0 = autotune batch, scatter mode, "
                                                        "tile and gather unroll on the first 64 frames")
    ap.add_argument("--scatter", type=int, default=0, help="0 auto, 1 atomic, 2 sorted, 3 staged")
    ap.add_argument("--tile", type=int, default=32, help="raster tile edge (with an explicit --batch)")
    ap.add_argument("--unroll", type=int, default=8, help="sorted-gather unroll (with an explicit --batch)")
    ap.add_argument("--small", type=int, default=48, help="single-lane triangle box area (with an explicit --batch)")
    ap.add_argument("--gwaves", type=int, default=8, help="gather grid waves per CU (with an explicit --batch)")
    ap.add_argument("--learned-site", type=int, default=0, choices=[0, 1],
                    help="learned weight: 0 its own pass, 1 inside the gather (with an explicit --batch)")
    ap.add_argument("--weighting", type=int, default=0,
                    help="0 w^(P), 1 w^(I), 2 learned (a seeded, untrained network), 3 mixed w^(P)/w^(I)")
    ap.add_argument("--layout", default="nhwc", choices=["nchw", "nhwc"])
    ap.add_argument("--input", default="f32", choices=["f32", "fp8"],
                    help="headline input: FP32 probabilities, or OCP E4M3 codes with a per-pixel FP32 scale")
    ap.add_argument("--cpu-frames", type=int, default=200)
    ap.add_argument("--cpu-frames-1t", type=int, default=16, help="frames of the one-thread oracle timing")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the NCHW / FP8 / w^(I) / learned throughput legs")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the label-accuracy report")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-scene batched graph leg")
    ap.add_argument("--no-isolated", action="store_true",
                    help="skip timing the gather alone (roofline_isolated); for profiling the headline launches")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding frames across GPUs (a "
                                   "reduce-scatter of the texel array) is designed but not implemented",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2111_11103_amd import scenes as S
    from paper_2111_11103_amd import semfuse as sf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)
        return
    t0 = time.time()
    log(f"[bench] generating workload: {args.frames} frames 640x480 c=40 on {torch.cuda.get_device_name(0)}")
    work = S.config2(device="cuda", n_frames=args.frames)
    sc = work.scene
    probs_nchw = work.probs
    probs = probs_nchw.to(memory_format=torch.channels_last) if args.layout == "nhwc" else probs_nchw
    torch.cuda.synchronize()
    log(f"[bench] workload ready in {time.time() - t0:.1f} s: T={sc.n_faces} V={sc.vertices.shape[0]}")
    F, c, H, W = probs.shape
    cams = torch.as_tensor(work.cams, device=dev)
    mesh = sf.Mesh(torch.as_tensor(sc.vertices, device=dev), torch.as_tensor(sc.faces, device=dev),
                   n_classes=c, s=work.s, scheme=work.scheme, keep_weights=False)
    l_out = torch.empty((F, H, W), dtype=torch.int32, device=dev)
    labels_img = torch.empty((F, H, W), dtype=torch.uint8, device=dev)
    tex = torch.empty((mesh.n_texels, c), dtype=torch.float32, device=dev)
    lab = torch.empty(mesh.n_texels, dtype=torch.uint8, device=dev)
    valid = work.valid
    L = sf.lib()
    head_probs, head_scale = probs, None
    if args.input == "fp8":
        # quantised in chunks, in the layout of the FP32 input
        head_probs = torch.empty((F, c, H, W), dtype=torch.uint8, device=dev)
        if args.layout == "nhwc":
            head_probs = head_probs.to(memory_format=torch.channels_last)
        head_scale = torch.empty((F, H, W), dtype=torch.float32, device=dev)
        for f0 in range(0, F, 50):
            qq, ss = S.quantize_fp8(probs[f0:f0 + 50])
            head_probs[f0:f0 + 50] = qq
            head_scale[f0:f0 + 50] = ss
        del qq, ss
    if args.weighting == sf.W_LEARNED:
        mesh.bind_mlp(sf.WeightMLP("cuda", seed=0))
    tuning = None
    if args.batch <= 0:
        from paper_2111_11103_amd import tune
        tuning = tune.autotune(mesh, cams, head_probs, scale=head_scale, valid=valid, weighting=args.weighting,
                               probe_frames=64, log=log)
        args.batch, args.scatter = int(tuning["batch"]), int(tuning["scatter_mode"])
    else:
        mesh.set_tuning(args.tile, args.unroll, args.small, args.gwaves, args.learned_site)

    def make_step(p, weighting, scale=None, batch=args.batch, scatter=args.scatter):
        ws = mesh.frame_ws(H, W, batch, weighting, scatter, probs=p)

        def step():
            mesh.reset()
            mesh.fuse_frames(cams, p, scale=scale, valid=valid, weighting=weighting, l_out=l_out, batch=batch,
                             scatter_mode=scatter, ws=ws)
            sf._check(L.lf_finalize(mesh._h, sf._ptr(tex), sf.F32, sf._ptr(lab), sf._stream()))
            mesh.render_labels(lab, l=l_out, valid=valid, out=labels_img)
        return step, ws

    def timed(step, steps, warmup, tag):
        for i in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"[bench] {tag}: warmup {i + 1}/{warmup} done")
        prof = Prof()
        sf._check(L.lf_profile_enable(mesh._h, 1))
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t_start
        sf._check(L.lf_profile_read(mesh._h, C.byref(prof)))
        sf._check(L.lf_profile_enable(mesh._h, 0))
        log(f"[bench] {tag}: {steps} steps, {1000 * t_total / steps:.3f} ms/step")
        return t_total, prof

    step, ws = make_step(head_probs, args.weighting, scale=head_scale)
    t_total, prof = timed(step, args.steps, args.warmup, "headline")
    ms_step = 1000.0 * t_total / args.steps
    npx = F * H * W
    value = npx / (t_total / args.steps)
    stage_ms = {STAGES[k]: prof.ms[k] / args.steps for k in range(8) if prof.launches[k]}
    log(f"[bench] {value / 1e9:.3f} G px/s; per stage ms/step {stage_ms}")

    # roofline of the dominant kernel (the gather, stage 2): algorithmic bytes
    # = every pixel's c class values + its valid byte, per launch (one launch
    # per batch of frames); duration = mean of the HIP-event-timed launches
    in_bytes = {torch.float32: 4, torch.uint8: 1}[head_probs.dtype]
    per_px = c * in_bytes + 1 + (4 if head_scale is not None else 0)     # classes, validity byte, FP8 scale
    launches = prof.launches[2]
    scat_ms = prof.ms[2] / launches
    px_per_launch = npx * args.steps / launches
    achieved = px_per_launch * per_px / (scat_ms * 1e-3) / 1e9
    # texel rows each launch reads and writes back once (distinct valid rows per batch)
    rows = 0
    for f0 in range(0, F, args.batch):
        lb = l_out[f0:f0 + args.batch]
        rows += int(torch.unique(lb[(lb >= 0) & (valid[f0:f0 + args.batch] != 0)]).numel())
    n_batches = (F + args.batch - 1) // args.batch
    rows_per_launch = rows / n_batches
    rmw_bytes = rows_per_launch * 2 * c * 4
    tpx = measured_traffic({"batch": args.batch, "scatter_mode": args.scatter, **mesh.get_tuning()})
    traffic = None if tpx is None else tpx * px_per_launch     # HBM bytes per launch (counters, calibrated)
    b_min = npx * per_px + mesh.n_texels * c * 4
    # B_alg: B_min plus the per-frame read-modify-write of every texel row a
    # frame touches (D_f distinct valid rows of frame f), as the update loop
    # of Section 3.3.2 states it frame by frame
    d_f = [int(torch.unique(l_out[f][(l_out[f] >= 0) & (valid[f] != 0)]).numel()) for f in range(F)]
    b_alg = b_min + sum(d_f) * 2 * c * 4
    log(f"[bench] gather {scat_ms:.3f} ms/launch; {rows_per_launch:.0f} rows per launch; "
        f"B_min {b_min / 1e9:.2f} GB -> {b_min / (t_total / args.steps) / 1e9:.0f} GB/s whole step; "
        f"B_alg {b_alg / 1e9:.2f} GB (mean D_f {sum(d_f) / F:.0f})")
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "fused pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"room mesh {sc.n_faces} triangles, SPLIT s=3 ({mesh.n_texels} texels), "
                               f"{F} frames {W}x{H}, c={c}, "
                               + ("FP32 " if args.input == "f32" else "FP8 E4M3 (per-pixel FP32 scale) ")
                               + f"{args.layout.upper()} probabilities, "
                               f"weighting {['w^(P)', 'w^(I)', 'learned', 'mixed'][args.weighting]}",
                   "frames": F, "H": H, "W": W, "classes": c, "triangles": sc.n_faces, "texels": mesh.n_texels,
                   "batch": args.batch, "scatter_mode": args.scatter, "frame_ws_bytes": ws.numel(),
                   "tuning": mesh.get_tuning(), "autotuned": tuning is not None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_bucket_gather16", "kernel_ms": scat_ms, "launches": launches,
                     "bytes_per_px": per_px, "px_per_launch": px_per_launch,
                     "row_rmw_bytes_per_launch": rmw_bytes,
                     "achieved_incl_row_rmw": (px_per_launch * per_px + rmw_bytes) / (scat_ms * 1e-3) / 1e9},
        "step_hbm_frac": b_min / (t_total / args.steps) / 1e9 / HBM_PEAK_GBS,
        "step_bytes": {"b_min": b_min, "b_alg": b_alg, "distinct_rows_per_frame": sum(d_f) / F,
                       "b_min_frac": b_min / (t_total / args.steps) / 1e9 / HBM_PEAK_GBS,
                       "b_alg_frac": b_alg / (t_total / args.steps) / 1e9 / HBM_PEAK_GBS},
        "stage_ms_per_step": stage_ms,
    }

    probe = device_probe(dev)
    result["device_probe"] = probe
    result["roofline"]["measured_copy_gbs"] = probe["copy_gbs"]
    result["roofline"]["frac_of_measured_copy"] = achieved / probe["copy_gbs"]
    log(f"[bench] device probe: {probe}")

    # the same gather launches without the concurrent raster (gathers on the
    # caller's stream, one batch after another) on a grid for the whole device
    def isolated_leg(result):
        saved = mesh.get_tuning()
        mesh.set_overlap(False)
        mesh.set_tuning(saved["tile"], saved["gather_unroll"], saved["small_px"], ISO_GATHER_WAVES)
        st_iso = make_step(head_probs, args.weighting, scale=head_scale)[0]
        tt_iso, pr_iso = timed(st_iso, 2, 1, "gather alone")
        mesh.set_overlap(True)
        mesh.set_tuning(**saved)
        iso_ms = pr_iso.ms[2] / pr_iso.launches[2]
        iso_px = npx * 2 / pr_iso.launches[2]
        iso_gbs = iso_px * per_px / (iso_ms * 1e-3) / 1e9
        result["roofline_isolated"] = {"kernel": "k_bucket_gather16", "bound": "hbm", "achieved": iso_gbs,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": iso_gbs / HBM_PEAK_GBS,
                                       "kernel_ms": iso_ms, "gather_waves": ISO_GATHER_WAVES,
                                       "step_value_without_overlap": 2 * npx / tt_iso}
        result["roofline_isolated"]["frac_of_measured_copy"] = iso_gbs / probe["copy_gbs"]
        log(f"[bench] gather alone: {iso_ms:.3f} ms/launch, {iso_gbs:.0f} GB/s algorithmic "
            f"({iso_gbs / HBM_PEAK_GBS:.1%}); whole step without overlap {2 * npx / tt_iso / 1e9:.2f} G px/s")

    if args.no_isolated:
        result["roofline_isolated"] = None
    else:
        isolated_leg(result)

    if not args.no_forms:
        forms = {}
        legs = [("nchw", lambda: make_step(probs_nchw, 0, scatter=0)[0], None)]
        legs.append(("w_image", lambda: make_step(probs, 1)[0], None))
        mlp_holder = {}

        def learned_step():
            mlp_holder["mlp"] = sf.WeightMLP("cuda", seed=0)
            mesh.bind_mlp(mlp_holder["mlp"])
            if tuning is None:
                return make_step(probs, sf.W_LEARNED)[0]
            # the learned weight's gather is the longer stream: its own tuning
            from paper_2111_11103_amd import tune
            mlp_holder["saved"] = mesh.get_tuning()
            t = tune.autotune(mesh, cams, probs, valid=valid, weighting=sf.W_LEARNED, probe_frames=64, log=log)
            mlp_holder["tuning"] = t
            return make_step(probs, sf.W_LEARNED, batch=int(t["batch"]), scatter=int(t["scatter_mode"]))[0]
        legs.append(("learned", learned_step, None))
        for name, mk, _ in legs:
            st = mk()
            tt, pr = timed(st, 2, 1, name)
            forms[name] = {"value": 2 * npx / tt, "ms_per_step": 1000 * tt / 2,
                           "stage_ms_per_step": {STAGES[k]: pr.ms[k] / 2 for k in range(8) if pr.launches[k]}}
        if "tuning" in mlp_holder:
            forms["learned"]["tuning"] = {k: mlp_holder["tuning"][k] for k in
                                          ("batch", "scatter_mode", "tile", "small_px", "gather_unroll", "gather_waves",
                                           "learned_in_gather")}
            mesh.set_tuning(**mlp_holder["saved"])
        mesh.bind_mlp(None)
        # the paper's texture resolution: a_t from the worst-case frame, s_t =
        # max(1, ceil(0.2 sqrt(a_t))), SQUARE texels (Section 3.1)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        area = mesh.triangle_max_pixels(cams, H, W, batch=32)
        s_face = sf.texel_resolution(area, 0.2)
        ev1.record()
        ev1.synchronize()
        area_ms = ev0.elapsed_time(ev1)
        mesh_g = sf.Mesh(torch.as_tensor(sc.vertices, device=dev), torch.as_tensor(sc.faces, device=dev),
                         n_classes=c, scheme=sf.SQUARE, s_face=s_face, keep_weights=False)
        mesh_g.set_tuning(**mesh.get_tuning())
        tex_g = torch.empty((mesh_g.n_texels, c), dtype=torch.float32, device=dev)
        lab_g = torch.empty(mesh_g.n_texels, dtype=torch.uint8, device=dev)
        ws_g = mesh_g.frame_ws(H, W, args.batch, 1, args.scatter, probs=probs)

        def gamma_step():
            mesh_g.reset()
            mesh_g.fuse_frames(cams, probs, valid=valid, weighting=1, l_out=l_out, batch=args.batch,
                               scatter_mode=args.scatter, ws=ws_g)
            sf._check(L.lf_finalize(mesh_g._h, sf._ptr(tex_g), sf.F32, sf._ptr(lab_g), sf._stream()))
            mesh_g.render_labels(lab_g, l=l_out, valid=valid, out=labels_img)
        gamma_step()
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(2):
            gamma_step()
        torch.cuda.synchronize()
        tg = (time.perf_counter() - tg) / 2
        forms["square_gamma0.2_w_image"] = {"value": npx / tg, "ms_per_step": 1000 * tg,
                                            "texels": mesh_g.n_texels, "area_pass_ms": area_ms,
                                            "max_s": int(s_face.max())}
        del mesh_g, tex_g, lab_g, ws_g
        # FP8 E4M3 input with a per-pixel scale (quantised in chunks, channels-last)
        q = torch.empty((F, c, H, W), dtype=torch.uint8, device=dev).to(memory_format=torch.channels_last)
        qs = torch.empty((F, H, W), dtype=torch.float32, device=dev)
        for f0 in range(0, F, 50):
            qq, ss = S.quantize_fp8(probs[f0:f0 + 50])
            q[f0:f0 + 50] = qq
            qs[f0:f0 + 50] = ss
        del qq, ss
        st = make_step(q, 0, scale=qs)[0]
        tt, pr = timed(st, 2, 1, "fp8")
        forms["fp8_input"] = {"value": 2 * npx / tt, "ms_per_step": 1000 * tt / 2,
                              "stage_ms_per_step": {STAGES[k]: pr.ms[k] / 2 for k in range(8) if pr.launches[k]}}
        del q, qs
        result["forms"] = forms
        log(f"[bench] forms: " + ", ".join(f"{k} {v['value'] / 1e9:.2f} G px/s" for k, v in forms.items()))

    if not args.no_cpu:
        log(f"[bench] CPU oracle on {args.cpu_frames} frames (all threads) and {args.cpu_frames_1t} (one thread) ...")
        result["cpu_baseline"], l_o, A_o = cpu_baseline(work, min(args.cpu_frames, F), min(args.cpu_frames_1t, F))
        if head_scale is None and args.weighting == 0:
            result["check"] = result_check(mesh, cams, head_probs, valid, l_o, A_o, args.batch, args.scatter)
            log(f"[bench] result check against the oracle: {result['check']}")
        del l_o, A_o
    else:
        result["cpu_baseline"] = None

    if not args.no_accuracy:
        result["accuracy"], mlp = accuracy_report(log)
        result["learned_at_scale"] = learned_scale_report(mlp, log)
        result["sweeps"] = weight_and_frame_sweeps(log)
        del mlp

    if not args.no_batched:
        torch.cuda.empty_cache()
        result["batched"] = batched_report(log)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
