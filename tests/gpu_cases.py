"""Shared helpers of the GPU parity tests: build a workload, run it through the
HIP library (C-ABI) and through the CPU oracle on the same bytes, compare."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf

REL_TOL = 1e-5          # relative tolerance on fused distributions (binary32 accumulation vs binary64)


def say(*a):
    print(*a, flush=True)


def to_dev(x, dtype=None):
    t = torch.as_tensor(x)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_mesh(scene_or_VF, s, scheme, c, aggregator=sf.AGG_SUM, s_face=None, z_near=0.05):
    V, F = scene_or_VF
    return sf.Mesh(to_dev(V, torch.float32), to_dev(F, torch.int32), n_classes=c, s=s, scheme=scheme,
                   aggregator=aggregator, s_face=None if s_face is None else to_dev(s_face, torch.int32),
                   z_near=z_near)


def oracle_mesh(V, F, s, scheme, s_face=None):
    return oracle.Mesh(V, F, s=s, scheme=scheme, s_face=s_face)


def compare_raster(gm, om, cams, H, W, z_near=0.05):
    """Bit-exact triangle ids, texel rows and depths on every pixel."""
    out = gm.rasterize(to_dev(cams, torch.float32), H, W)
    torch.cuda.synchronize()
    tri_g = out["tri"].cpu().numpy()
    l_g = out["l"].cpu().numpy()
    z_g = out["z"].cpu().numpy()
    tri_o, l_o = om.raster_frames(cams, H, W, z_near=z_near)
    for f in range(len(cams)):
        d = np.argwhere(tri_g[f] != tri_o[f])
        assert d.size == 0, f"frame {f}: {len(d)} triangle-id mismatches, first {d[:5].tolist()}"
        d = np.argwhere(l_g[f] != l_o[f])
        assert d.size == 0, f"frame {f}: {len(d)} texel-row mismatches, first {d[:5].tolist()}"
    # depth of the winning fragment, bit for bit (NaN where nothing is hit)
    _, _, z0 = om.raster(cams[0], H, W, z_near)
    assert np.array_equal(z_g[0].view(np.uint32), z0.view(np.uint32))
    return tri_o, l_o


def compare_fused(A_gpu, A_or, W_or=None, aggregator=sf.AGG_SUM, rel=REL_TOL):
    """Per-entry relative error of the binary32 accumulator against binary64."""
    A_gpu = A_gpu.astype(np.float64)
    if aggregator == sf.AGG_MUL:
        # log domain: |dA| <= rel * |A| (+ tiny absolute slack for near-zero logs)
        err = np.abs(A_gpu - A_or)
        bad = err > rel * np.abs(A_or) + 1e-6
    else:
        err = np.abs(A_gpu - A_or)
        bad = err > rel * np.abs(A_or)
    n_bad = int(bad.sum())
    worst = float((err / np.maximum(np.abs(A_or), 1e-300)).max()) if A_or.size else 0.0
    assert n_bad == 0, f"{n_bad} accumulator entries beyond {rel} relative (worst {worst:.3g})"
    return worst


def compare_labels(lab_gpu, P_or, lab_or, rel=REL_TOL):
    """Labels equal wherever the oracle's top-2 margin exceeds the tolerance."""
    srt = np.sort(P_or, axis=1)
    p1, p2 = srt[:, -1], srt[:, -2] if P_or.shape[1] > 1 else np.zeros(len(P_or))
    clear = (lab_or == 255) | ((p1 - p2) > rel * p1)
    mism = (lab_gpu != lab_or) & clear
    assert not mism.any(), f"{int(mism.sum())} labels differ on texels with a clear margin"
    return int((~clear).sum())


def compare_normalized(P_gpu, P_or, rel=REL_TOL):
    err = np.abs(P_gpu.astype(np.float64) - P_or)
    bad = err > rel * np.abs(P_or)
    assert not bad.any(), f"{int(bad.sum())} normalised entries beyond {rel} relative"
