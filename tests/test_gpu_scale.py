"""Parity at the large shapes the benchmark runs, through the C-ABI:

* the learned-form scene shape: a 2M-triangle room, SPLIT s = 4 (32M texels),
  frames of 1296x968, c = 40, channels-last FP32 through lf_fuse_frames
  (bit-exact triangle ids and texel rows, fused rows within 1e-5), plus the
  raster with 16-pixel tiles (81 x 61 tiles: more than the binning's LDS
  tile counters hold, so binning reserves list slots with global atomics);
* the headline launch exactly as the benchmark tunes it (c = 40, 64 frames
  per batch, 32-pixel tiles, single-lane boxes up to 96 px, gather unroll 8,
  8 gather waves per CU) over three batches, the last one ragged;
* a captured HIP graph of two c = 40 scenes (the grouped texel-sorted gather
  with its second stream inside the graph), one of them 1296x968 with 16-pixel
  tiles, replayed twice.

Oracle rows are compared on the texel rows the frames touch (the oracle's
binary64 accumulator is indexed by a compact renumbering of those rows);
every other row must stay exactly zero on the device."""
import numpy as np
import pytest
import torch

import oracle
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf
from tests.gpu_cases import compare_fused, compare_labels, compare_normalized, compare_raster, say, to_dev

pytestmark = pytest.mark.gpu


def _compact_oracle(om, c, l_o, probs_np, valid_np, weighting=oracle.W_PIXEL):
    """binary64 fusion on the touched rows only: (rows, A [n_rows, c], W [n_rows])."""
    sel = (l_o >= 0) & (valid_np != 0)
    rows = np.unique(l_o[sel])
    # (an invalid pixel may land on a row outside the list: the oracle skips it unread)
    lc = np.where(l_o >= 0, np.searchsorted(rows, np.maximum(l_o, 0)), -1).astype(np.int32)
    A, W = oracle.fuse(len(rows), c, lc, probs_np, valid_np, weighting=weighting)
    return rows, A, W


def _check_rows(accum, rows, A_o):
    """Touched rows within 1e-5 relative of binary64, all other rows exactly zero."""
    idx = torch.from_numpy(rows.astype(np.int64)).cuda()
    compare_fused(accum[idx].cpu().numpy(), A_o)
    rest = accum.clone()
    rest[idx] = 0
    assert float(rest.abs().max()) == 0.0, "rows no pixel touched were written"


@pytest.fixture(scope="module")
def big_scene():
    say("[case] 2M-triangle room, SPLIT s=4 (32M texels), 1296x968, c=40")
    sc = S.config2_scene(seed=0, target_tris=2_000_000)
    H, W = 968, 1296
    cams = S.random_walk_cameras(sc, 24, W, H, seed=0)
    probs, valid, _ = S.frame_inputs(sc, cams, H, W, margin=3.0, sigma=2.0, blob_frac=0.15, invalid_frac=0.05,
                                     seed=0, device="cuda", chunk=8)
    return sc, cams, H, W, probs, valid


def test_learned_form_scene_shape(big_scene):
    """24 frames (three batches of 8) of 1296x968 on the 2M-triangle, 32M-texel
    mesh: every triangle id, texel row and the first frame's depths equal the
    oracle's; every touched row of the fused texture within 1e-5 relative
    (w^(P) and w^(I)); then 16-pixel tiles give the same renderer output."""
    sc, cams, H, W, probs, valid = big_scene
    om = oracle.Mesh(sc.vertices, sc.faces, s=4, scheme=oracle.SPLIT)
    gm = sf.Mesh(to_dev(sc.vertices, torch.float32), to_dev(sc.faces, torch.int32), n_classes=40, s=4,
                 scheme=sf.SPLIT, keep_weights=False)
    assert gm.n_texels == om.n_texels == 31963136
    say("  raster, 32-pixel tiles")
    _, l_o = compare_raster(gm, om, cams, H, W)
    cl = probs.to(memory_format=torch.channels_last)
    probs_np, valid_np = probs.cpu().numpy(), valid.cpu().numpy()
    for weighting in (sf.W_PIXEL, sf.W_IMAGE):
        say(f"  fuse 24 frames, batch 8, weighting {weighting}")
        gm.reset()
        l_out = torch.empty((len(cams), H, W), dtype=torch.int32, device="cuda")
        gm.fuse_frames(to_dev(cams, torch.float32), cl, valid=valid, weighting=weighting, l_out=l_out, batch=8)
        torch.cuda.synchronize()
        assert np.array_equal(l_out.cpu().numpy(), l_o)
        rows, A_o, _ = _compact_oracle(om, 40, l_o, probs_np, valid_np, weighting)
        say(f"  {len(rows)} touched rows")
        _check_rows(gm.accum, rows, A_o)
    say("  raster, 16-pixel tiles (81 x 61 tiles: binning through global atomics)")
    gm.set_tuning(16, 8, 48, 8)
    r = gm.rasterize(to_dev(cams[:6], torch.float32), H, W)
    torch.cuda.synchronize()
    assert np.array_equal(r["l"].cpu().numpy(), l_o[:6])


@pytest.fixture(scope="module")
def headline_work():
    say("[case] headline workload: 500k-triangle room, SPLIT s=3, 130 frames 640x480, c=40")
    return S.config2(device="cuda", n_frames=130)


def test_headline_launch_exactly(headline_work):
    """The benchmark's tuned headline launch on 130 frames (batches of 64, 64
    and 2): texel rows bit-exact, the fused texture within 1e-5 per entry,
    normalised texture and labels, and the rendered label images."""
    w = headline_work
    sc = w.scene
    F = len(w.cams)
    om = oracle.Mesh(sc.vertices, sc.faces, s=3, scheme=oracle.SPLIT)
    gm = sf.Mesh(to_dev(sc.vertices, torch.float32), to_dev(sc.faces, torch.int32), n_classes=40, s=3,
                 scheme=sf.SPLIT, keep_weights=False)
    gm.set_tuning(32, 8, 96, 8)
    cams = to_dev(w.cams, torch.float32)
    cl = w.probs.to(memory_format=torch.channels_last)
    l_out = torch.empty((F, w.H, w.W), dtype=torch.int32, device="cuda")
    say("  fuse (batch 64, sorted)")
    gm.fuse_frames(cams, cl, valid=w.valid, l_out=l_out, batch=64, scatter_mode=sf.SCATTER_SORTED)
    tex, lab = gm.finalize()
    img = gm.render_labels(lab, l=l_out, valid=w.valid)
    torch.cuda.synchronize()
    say("  oracle raster + fusion")
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    assert np.array_equal(l_out.cpu().numpy(), l_o)
    valid_np = w.valid.cpu().numpy()
    A_o, W_o = oracle.fuse(om.n_texels, 40, l_o, w.probs.cpu().numpy(), valid_np)
    compare_fused(gm.accum.cpu().numpy(), A_o)
    P_o, lab_o = oracle.finalize(A_o, W_o)
    compare_normalized(tex.cpu().numpy(), P_o)
    lab_g = lab.cpu().numpy()
    compare_labels(lab_g, P_o, lab_o)
    assert np.array_equal(img.cpu().numpy(), oracle.render(l_o, lab_g, valid_np))


def test_graph_c40_with_large_frames():
    """Two c = 40 scenes captured as one graph: 640x480 (batch 16, pool 16,
    32-pixel tiles) and 1296x968 (batch 8, pool 8, 16-pixel tiles); both go
    through the grouped texel-sorted gather on the library's second stream.
    Two replays with eager work between them, each checked against the
    oracle."""
    say("[case] captured graph, c=40, 640x480 + 1296x968 scenes")
    specs = [(1000, 60_000, 2, 480, 640, 16, 40, 32), (1001, 80_000, 1, 968, 1296, 8, 20, 16)]
    data = []
    for seed, T, s, H, W, pool, F, tile in specs:
        sc = S.config2_scene(seed=seed, target_tris=T)
        cams = S.random_walk_cameras(sc, F, W, H, seed=seed)
        probs, valid, _ = S.frame_inputs(sc, cams[:pool], H, W, margin=3.0, sigma=2.0, blob_frac=0.15,
                                         invalid_frac=0.05, seed=seed, device="cuda")
        om = oracle.Mesh(sc.vertices, sc.faces, s=s, scheme=oracle.SPLIT)
        _, l_o = om.raster_frames(cams, H, W)
        idx = np.arange(F) % pool
        valid_exp = valid.cpu().numpy()[idx]
        A_o, W_o = oracle.fuse(om.n_texels, 40, l_o, probs.cpu().numpy()[idx], valid_exp)
        P_o, lab_o = oracle.finalize(A_o, W_o)
        data.append(dict(sc=sc, cams=cams, H=H, W=W, s=s, pool=pool, tile=tile, probs=probs, valid=valid,
                         l_o=l_o, P_o=P_o, lab_o=lab_o, valid_exp=valid_exp))

    def jobs_of(batches):
        jobs = []
        for d, b in zip(data, batches):
            m = sf.Mesh(to_dev(d["sc"].vertices, torch.float32), to_dev(d["sc"].faces, torch.int32), n_classes=40,
                        s=d["s"], scheme=sf.SPLIT, keep_weights=False)
            m.set_tuning(d["tile"], 8, 96, 8)
            jobs.append(m.job(to_dev(d["cams"], torch.float32), d["probs"].to(memory_format=torch.channels_last),
                              valid=d["valid"], pool=d["pool"], batch=b, scatter_mode=sf.SCATTER_SORTED,
                              tex_dtype=torch.float32, images=True))
        return jobs

    def check(jobs, tag):
        torch.cuda.synchronize()
        for j, d in zip(jobs, data):
            assert np.array_equal(j.l.cpu().numpy(), d["l_o"]), f"{tag}: texel rows differ"
            compare_normalized(j.tex.cpu().numpy(), d["P_o"])
            lab = j.labels.cpu().numpy()
            compare_labels(lab, d["P_o"], d["lab_o"])
            assert np.array_equal(j.images.cpu().numpy(), oracle.render(d["l_o"], lab, d["valid_exp"])), tag

    jobs = jobs_of((16, 8))
    g = sf.Graph(jobs)
    eager = jobs_of((7, 5))
    for rep in range(2):
        for j in jobs:
            j.labels.fill_(77)
            j.tex.fill_(-1.0)
            j.images.fill_(77)
        g.launch()
        check(jobs, f"replay {rep}")
        sf.fuse_batch(eager)
        check(eager, f"eager after replay {rep}")
