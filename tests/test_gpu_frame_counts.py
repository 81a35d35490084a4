"""w^(I) and the mixed weight (Section 3.2.2) on the grouped texel-sorted
gather, which counts each texel row's observations per frame of the batch
itself (LDS counters) instead of reading per-frame counts written by the
raster: parity with the oracle for ragged batches, one-frame batches, FP8
input, planar input through the staged path, rows of several hundred thousand
observations, and a frame-innermost layout whose frames cannot be recovered
from the stored offsets (that one takes the per-frame count array).  Also the
E4M3 scales the same gather reads from the input's scale array."""
import numpy as np
import pytest
import torch

import oracle
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf
from tests.gpu_cases import (compare_fused, compare_labels, compare_normalized, gpu_mesh, oracle_mesh, say,
                             to_dev)

pytestmark = pytest.mark.gpu

C = 16   # a multiple of 4 up to 64: the grouped gather


@pytest.fixture(scope="module")
def case():
    say("[case] config-1 scene (2,100 triangles, 20 frames 160x120) with c=16 probabilities")
    w = S.config1(device="cpu")
    g = torch.Generator().manual_seed(1234)
    probs = torch.softmax(2.0 * torch.randn((w.cams.shape[0], C, w.H, w.W), generator=g), 1)
    sc = w.scene
    om = oracle_mesh(sc.vertices, sc.faces, 1, oracle.SPLIT)
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    return w, probs, om, l_o


def _check_wsum(gm, W_ref, l_o, valid):
    # the weight sum of a row: binary32 adds, one per observation
    seen = (l_o >= 0) & (valid != 0)
    n_obs = np.bincount(l_o[seen], minlength=W_ref.shape[0]).astype(np.float64)
    assert np.all(np.abs(gm.wsum.cpu().numpy() - W_ref) <= (n_obs + 1) * 2.0 ** -24 * W_ref)


@pytest.mark.parametrize("layout", ["nhwc", "staged"])
@pytest.mark.parametrize("batch", [1, 7, 20])
def test_image_weight_counted_in_gather(case, layout, batch):
    w, probs, om, l_o = case
    say(f"  w^(I), {layout}, batch {batch}")
    sc = w.scene
    valid = w.valid.numpy()
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
    x = probs.to(memory_format=torch.channels_last).cuda() if layout == "nhwc" else probs.cuda()
    mode = sf.SCATTER_SORTED if layout == "nhwc" else sf.SCATTER_STAGED
    gm.fuse_frames(to_dev(w.cams, torch.float32), x, valid=w.valid.cuda(), weighting=sf.W_IMAGE, batch=batch,
                   scatter_mode=mode)
    tex, lab = gm.finalize()
    torch.cuda.synchronize()
    A_o, W_o = oracle.fuse(om.n_texels, C, l_o, probs.numpy(), valid, weighting=sf.W_IMAGE)
    compare_fused(gm.accum.cpu().numpy(), A_o)
    _check_wsum(gm, W_o, l_o, valid)
    P_o, lab_o = oracle.finalize(A_o, W_o)
    compare_normalized(tex.cpu().numpy(), P_o)
    compare_labels(lab.cpu().numpy(), P_o, lab_o)


def test_mixed_weight_counted_in_gather(case):
    """w = (1 - a) + a / n fuses to (1 - a) A^(P) + a A^(I) by linearity."""
    w, probs, om, l_o = case
    sc = w.scene
    valid = w.valid.numpy()
    A_p, W_p = oracle.fuse(om.n_texels, C, l_o, probs.numpy(), valid, weighting=sf.W_PIXEL)
    A_i, W_i = oracle.fuse(om.n_texels, C, l_o, probs.numpy(), valid, weighting=sf.W_IMAGE)
    x = probs.to(memory_format=torch.channels_last).cuda()
    for alpha in (0.25, 1.0):
        say(f"  mixed weight alpha {alpha}")
        gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
        gm.set_weight_mix(alpha)
        gm.fuse_frames(to_dev(w.cams, torch.float32), x, valid=w.valid.cuda(), weighting=sf.W_MIX, batch=6,
                       scatter_mode=sf.SCATTER_SORTED)
        torch.cuda.synchronize()
        compare_fused(gm.accum.cpu().numpy(), (1 - alpha) * A_p + alpha * A_i)
        _check_wsum(gm, (1 - alpha) * W_p + alpha * W_i, l_o, valid)


def test_image_weight_fp8_counted_in_gather(case):
    w, probs, om, l_o = case
    say("  w^(I), channels-last FP8 E4M3 with per-pixel scale")
    sc = w.scene
    valid = w.valid.numpy()
    q, scale = S.quantize_fp8(probs)
    A8, _ = oracle.fuse(om.n_texels, C, l_o, q.numpy(), valid, weighting=sf.W_IMAGE, scale=scale.numpy())
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
    gm.fuse_frames(to_dev(w.cams, torch.float32), q.to(memory_format=torch.channels_last).cuda(),
                   scale=scale.cuda(), valid=w.valid.cuda(), weighting=sf.W_IMAGE, batch=8,
                   scatter_mode=sf.SCATTER_SORTED)
    torch.cuda.synchronize()
    compare_fused(gm.accum.cpu().numpy(), A8)


def test_frame_innermost_layout_uses_count_array(case):
    """Storage [H][W][F][c]: the frame stride (c) is smaller than a frame's
    pixel offsets, so the frame of a stored offset is not offset / stride;
    the per-frame count array serves this layout, with the same result."""
    w, probs, om, l_o = case
    say("  w^(I), frame-innermost storage")
    sc = w.scene
    valid = w.valid.numpy()
    x = probs.permute(2, 3, 0, 1).contiguous().permute(2, 3, 0, 1).cuda()
    assert x.stride()[0] == C and x.stride()[1] == 1
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
    gm.fuse_frames(to_dev(w.cams, torch.float32), x, valid=w.valid.cuda(), weighting=sf.W_IMAGE, batch=7,
                   scatter_mode=sf.SCATTER_SORTED)
    torch.cuda.synchronize()
    A_o, W_o = oracle.fuse(om.n_texels, C, l_o, probs.numpy(), valid, weighting=sf.W_IMAGE)
    compare_fused(gm.accum.cpu().numpy(), A_o)
    _check_wsum(gm, W_o, l_o, valid)


def test_image_weight_on_very_long_rows():
    """Two triangles with one texel each fill three 640x480 frames: each row
    holds ~460k observations, ~150k per frame, with a random validity mask."""
    say("[case] two-texel wall, 3 frames 640x480, c=4, w^(I)")
    fx, cx, cy = 512.0, 320.0, 240.0
    V = np.array([[-3, -2.5, 2], [3, -2.5, 2], [3, 2.5, 2], [-3, 2.5, 2]], np.float32)
    F_ = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    cams = np.array([[fx, fx, cx, cy, 1, 0, 0, 0, 1, 0, 0, 0, 1, tx, ty, 0]
                     for tx, ty in ((0.0, 0.0), (0.1, 0.0), (0.0, 0.1))], np.float32)
    gen = torch.Generator().manual_seed(5)
    probs = torch.softmax(torch.randn((3, 4, 480, 640), generator=gen), 1)
    valid = (torch.rand((3, 480, 640), generator=gen) > 0.2).to(torch.uint8)
    om = oracle_mesh(V, F_, 1, oracle.SPLIT)
    _, l_o = om.raster_frames(cams, 480, 640)
    assert om.n_texels == 2 and (l_o >= 0).all()
    A_o, W_o = oracle.fuse(om.n_texels, 4, l_o, probs.numpy(), valid.numpy(), weighting=sf.W_IMAGE)
    for batch in (3, 2):
        gm = gpu_mesh((V, F_), 1, oracle.SPLIT, 4)
        gm.fuse_frames(to_dev(cams), probs.to(memory_format=torch.channels_last).cuda(), valid=valid.cuda(),
                       weighting=sf.W_IMAGE, batch=batch, scatter_mode=sf.SCATTER_SORTED)
        torch.cuda.synchronize()
        compare_fused(gm.accum.cpu().numpy(), A_o)
        _check_wsum(gm, W_o, l_o, valid.numpy())
    # every frame adds weight 1 to each texel it sees: W = number of frames
    assert np.allclose(W_o, 3.0)


@pytest.mark.parametrize("layout", ["nhwc", "frame_innermost"])
def test_fp8_scales_read_by_gather(case, layout):
    """E4M3 input on the grouped gather: with pixels dense in the input
    (channels-last) the gather reads each observation's scale from the
    [F][H][W] scale array itself; the frame-innermost layout keeps the
    per-entry scales written by the fill.  Both equal the oracle."""
    w, probs, om, l_o = case
    say(f"  FP8 w^(P), {layout}")
    sc = w.scene
    valid = w.valid.numpy()
    q, scale = S.quantize_fp8(probs)
    A8, _ = oracle.fuse(om.n_texels, C, l_o, q.numpy(), valid, scale=scale.numpy())
    if layout == "nhwc":
        x = q.to(memory_format=torch.channels_last).cuda()
    else:
        x = q.permute(2, 3, 0, 1).contiguous().permute(2, 3, 0, 1).cuda()
    for batch in (7, 1):
        gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
        gm.fuse_frames(to_dev(w.cams, torch.float32), x, scale=scale.cuda(), valid=w.valid.cuda(), batch=batch,
                       scatter_mode=sf.SCATTER_SORTED)
        torch.cuda.synchronize()
        compare_fused(gm.accum.cpu().numpy(), A8)


def test_large_batches_and_pooled_fp8(case):
    """The 20 frames repeated 15 times (300 frames): by linearity the fused
    sums are 15 times those of the 20 distinct frames (w^(I) weights repeat
    with their frames).  Batches of 300 frames exceed the gather's 256 frame
    counters, so w^(I) takes the per-frame count array; batches of 64 count
    in the gather.  The same 300 frames as a scene job over an input pool of
    the 20 FP8 frames (frame f reads input f % 20): the gather reads each
    scale at the pooled input frame."""
    w, probs, om, l_o = case
    sc = w.scene
    valid = w.valid.numpy()
    rep = 15
    cams = to_dev(np.concatenate([w.cams] * rep), torch.float32)
    A_o, W_o = oracle.fuse(om.n_texels, C, l_o, probs.numpy(), valid, weighting=sf.W_IMAGE)
    x = probs.cuda().repeat(rep, 1, 1, 1).contiguous(memory_format=torch.channels_last)
    v = w.valid.cuda().repeat(rep, 1, 1)
    for batch in (300, 64):
        say(f"  w^(I), 300 frames, batch {batch}")
        gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
        gm.fuse_frames(cams, x, valid=v, weighting=sf.W_IMAGE, batch=batch, scatter_mode=sf.SCATTER_SORTED)
        torch.cuda.synchronize()
        compare_fused(gm.accum.cpu().numpy(), rep * A_o)
    del x, v
    say("  FP8 w^(P), 300 frames from a pool of 20, batch 64")
    q, scale = S.quantize_fp8(probs)
    A8, _ = oracle.fuse(om.n_texels, C, l_o, q.numpy(), valid, scale=scale.numpy())
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, C)
    job = gm.job(cams, q.to(memory_format=torch.channels_last).cuda(), scale=scale.cuda(), valid=w.valid.cuda(),
                 pool=len(w.cams), batch=64, scatter_mode=sf.SCATTER_SORTED)
    sf.fuse_batch([job])
    torch.cuda.synchronize()
    compare_fused(gm.accum.cpu().numpy(), rep * A8)
