"""Out-of-core aggregation (Section 3.3.2: the aggregator also runs where the
texture does not fit the GPU): the texture is fused a texel-row window at a
time into a window-sized device buffer, through the C-ABI (lf_set_window),
and the windows together must equal the oracle's whole texture.  Windows
much smaller than the texture, a ragged last window, the texel-sorted and
the atomic scatter, w^(P) / w^(I), and a mesh loaded with no whole-texture
accumulator at all."""
import numpy as np
import pytest
import torch

import oracle
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf
from tests.gpu_cases import compare_fused, compare_labels, compare_normalized, gpu_mesh, oracle_mesh, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg():
    say("[case] windowed fusion: config-1 room, SPLIT s=2 (4,200 texels), c=13 and c=16")
    w = S.config1(device="cpu")
    om = oracle_mesh(w.scene.vertices, w.scene.faces, 2, oracle.SPLIT)
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    return w, om, l_o


@pytest.mark.parametrize("weighting", [sf.W_PIXEL, sf.W_IMAGE])
@pytest.mark.parametrize("scatter,layout", [(sf.SCATTER_SORTED, "nhwc"), (sf.SCATTER_ATOMIC, "nchw")])
def test_windows_equal_whole_texture(cfg, weighting, scatter, layout):
    w, om, l_o = cfg
    sc = w.scene
    c = 16                                  # grouped texel-sorted gather on the sorted path
    g = torch.Generator().manual_seed(11)
    probs = torch.softmax(2.0 * torch.randn((len(w.cams), c, w.H, w.W), generator=g), 1)
    valid = w.valid
    A_o, W_o = oracle.fuse(om.n_texels, c, l_o, probs.numpy(), valid.numpy(), weighting=weighting)
    P_o, lab_o = oracle.finalize(A_o, W_o)
    x = probs.to(memory_format=torch.channels_last).cuda() if layout == "nhwc" else probs.cuda()
    gm = gpu_mesh((sc.vertices, sc.faces), 2, oracle.SPLIT, c)
    cams = to_dev(w.cams, torch.float32)
    for rows in (1000, 1537):
        say(f"  windows of {rows} rows, weighting {weighting}, scatter {scatter}")
        tex, lab = gm.fuse_windowed(cams, x, window_rows=rows, valid=valid.cuda(), weighting=weighting, batch=8,
                                    scatter_mode=scatter)
        compare_normalized(tex.numpy(), P_o)
        lab_g = lab.cpu().numpy()
        compare_labels(lab_g, P_o, lab_o)
        # the label images read the whole label array
        img = gm.render_labels(lab, l=to_dev(l_o, torch.int32), valid=valid.cuda())
        assert np.array_equal(img.cpu().numpy(), oracle.render(l_o, lab_g, valid.numpy()))
    # the whole-texture state is back: an ordinary fusion fills the load-time accumulator
    gm.reset()
    gm.fuse_frames(cams, x, valid=valid.cuda(), weighting=weighting, batch=8, scatter_mode=scatter)
    torch.cuda.synchronize()
    compare_fused(gm.accum.cpu().numpy(), A_o)


def test_window_accumulator_rows_and_no_whole_texture(cfg):
    """One explicit window in the middle of the texture: its buffer holds
    exactly the oracle's rows of that range (1e-5), nothing else is touched;
    a mesh loaded without a whole-texture accumulator fuses windows only."""
    w, om, l_o = cfg
    sc = w.scene
    probs = w.probs
    A_o, _ = oracle.fuse(om.n_texels, 13, l_o, probs.numpy(), w.valid.numpy(), weighting=oracle.W_IMAGE)
    cams = to_dev(w.cams, torch.float32)
    lo, n = 1234, 1500
    for whole in (True, False):
        gm = sf.Mesh(to_dev(sc.vertices, torch.float32), to_dev(sc.faces, torch.int32), n_classes=13, s=2,
                     scheme=sf.SPLIT, whole_texture=whole)
        if whole:
            gm.accum.fill_(7.0)                  # must stay untouched while the window is set
        acc = torch.full((n, 13), -1.0, device="cuda")
        wsum = torch.full((n,), -1.0, device="cuda")
        gm.set_window(lo, n, acc, wsum)
        gm.reset()
        for mode in (sf.SCATTER_ATOMIC, sf.SCATTER_SORTED):
            gm.reset()
            gm.fuse_frames(cams, probs.cuda() if mode == sf.SCATTER_ATOMIC
                           else probs.to(memory_format=torch.channels_last).cuda(),
                           valid=w.valid.cuda(), weighting=sf.W_IMAGE, batch=6, scatter_mode=mode)
            torch.cuda.synchronize()
            compare_fused(acc.cpu().numpy(), A_o[lo:lo + n])
        if whole:
            assert float((gm.accum - 7.0).abs().max()) == 0.0
            gm.set_window()
        else:
            with pytest.raises(sf.SemfuseError):
                gm.set_window()                   # there is no whole-texture accumulator to return to
    with pytest.raises(sf.SemfuseError):
        gm.set_window(om.n_texels - 10, 11, torch.empty((11, 13), device="cuda"))
