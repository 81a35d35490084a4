"""lf_fuse_frames_noalloc (fusion with the library's static per-device scratch
as the frame workspace) against lf_fuse_frames with a caller workspace, both
through the C-ABI on the same inputs: texel rows bit for bit, accumulators
within 1e-5 relative per entry, and both against the binary64 oracle.  Two
calls in a row on each mesh, the second with fewer frames of a smaller image
(the scratch keeps the first call's contents), for the texel-sorted gather
with w^(I) and the atomic scatter with w^(P); a call whose workspace exceeds
the scratch is refused before anything is launched."""
import numpy as np
import pytest
import torch

import oracle
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf
from tests.gpu_cases import compare_fused, gpu_mesh, oracle_mesh, say, to_dev

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def cfg():
    say("[case] no-alloc fusion: config-1 room, SPLIT s=2 (4,200 texels), 20 frames 160x120, c=13")
    w = S.config1(device="cpu")
    om = oracle_mesh(w.scene.vertices, w.scene.faces, 2, oracle.SPLIT)
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    return w, om, l_o


def _call(gm, noalloc, cams, probs, valid, weighting, scatter, batch):
    F, _, H, W = probs.shape
    l_out = torch.full((F, H, W), -7, dtype=torch.int32, device="cuda")
    gm.reset()
    fn = gm.fuse_frames_noalloc if noalloc else gm.fuse_frames
    fn(cams, probs, valid=valid, weighting=weighting, l_out=l_out, batch=batch, scatter_mode=scatter)
    torch.cuda.synchronize()
    return l_out.cpu().numpy(), gm.accum.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("weighting,scatter,layout", [(sf.W_IMAGE, sf.SCATTER_SORTED, "nhwc"),
                                                      (sf.W_PIXEL, sf.SCATTER_ATOMIC, "nchw")])
def test_noalloc_matches_workspace_call(cfg, weighting, scatter, layout):
    w, om, l_o = cfg
    sc = w.scene
    probs = w.probs.cuda()
    if layout == "nhwc":
        probs = probs.to(memory_format=torch.channels_last)
    valid = w.valid.cuda()
    cams = to_dev(w.cams, torch.float32)
    ref = gpu_mesh((sc.vertices, sc.faces), 2, oracle.SPLIT, 13)
    na = gpu_mesh((sc.vertices, sc.faces), 2, oracle.SPLIT, 13)
    # call 1: all 20 frames of 160 x 120; call 2: 7 frames cropped to 96 x 72
    # (same cameras, so the crop's rows are the full frames' rows there)
    calls = [(slice(0, 20), 120, 160, 8), (slice(3, 10), 72, 96, 3)]
    for i, (fs, H, W, batch) in enumerate(calls):
        say(f"  call {i + 1}: {fs.stop - fs.start} frames {W}x{H}, weighting {weighting}, scatter {scatter}")
        p = probs[fs, :, :H, :W]
        v = valid[fs, :H, :W]
        c = cams[fs]
        l_ref, A_ref = _call(ref, False, c, p, v, weighting, scatter, batch)
        l_na, A_na = _call(na, True, c, p, v, weighting, scatter, batch)
        lo = l_o[fs, :H, :W]
        assert np.array_equal(l_ref, lo), "workspace call: texel rows differ from the oracle"
        assert np.array_equal(l_na, lo), "no-alloc call: texel rows differ from the oracle"
        # the two device results, entry by entry
        bad = np.abs(A_na - A_ref) > REL * np.abs(A_ref)
        assert not bad.any(), f"{int(bad.sum())} entries of the no-alloc accumulator beyond {REL} of the workspace call's"
        # and both against binary64
        A_o, _ = oracle.fuse(om.n_texels, 13, np.ascontiguousarray(lo), p.cpu().numpy(), v.cpu().numpy(),
                             weighting=weighting)
        compare_fused(A_ref, A_o)
        compare_fused(A_na, A_o)
        assert (A_na != 0).any()


def test_noalloc_refuses_calls_beyond_the_scratch(cfg):
    """A 64-frame batch of 1296 x 968 needs 64 x 1.25M x 4 bytes of texel rows
    alone: refused with LF_ESIZE on the host, nothing launched."""
    w, _, _ = cfg
    sc = w.scene
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, 13)
    F, H, W = 64, 968, 1296
    probs = torch.empty((F, 13, H, W), dtype=torch.float32, device="cuda")
    cams = to_dev(np.repeat(w.cams[:1], F, axis=0), torch.float32)
    with pytest.raises(sf.SemfuseError) as e:
        gm.fuse_frames_noalloc(cams, probs, batch=64, scatter_mode=sf.SCATTER_ATOMIC)
    assert e.value.status == sf.LF_ESIZE
    assert "static scratch" in str(e.value)
