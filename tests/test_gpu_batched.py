"""Many scenes in one call and as one captured HIP graph, input pools, the
tuning knobs and the autotuner, against the binary64 oracle (through the
C-ABI)."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf
from paper_2111_11103_amd import tune
from tests.gpu_cases import compare_labels, compare_normalized, oracle_mesh, say, to_dev

pytestmark = pytest.mark.gpu


def _scene(seed, grid, n_frames, H, W, s, scheme, pool, fp8=False):
    sc = S.room_scene(seed=seed, room=(6.0, 5.0, 3.0), n_boxes=4 + seed % 3, n_classes=13, room_grid=grid, box_grid=1)
    cams = S.circle_cameras(sc, n_frames, W, H)
    n_in = pool if pool else n_frames
    probs, valid, _ = S.frame_inputs(sc, cams[:n_in], H, W, margin=3.0, sigma=1.5, blob_frac=0.1,
                                     invalid_frac=0.05, seed=seed)
    d = dict(sc=sc, cams=cams, H=H, W=W, s=s, scheme=scheme, pool=pool, probs=probs, valid=valid, fp8=fp8)
    if fp8:
        d["q"], d["scale"] = S.quantize_fp8(probs)
    return d


@pytest.fixture(scope="module")
def scenes():
    say("[case] batched: 3 scenes of uneven size (pool 8 / none / pool 4 FP8 channels-last)")
    out = [_scene(0, 13, 20, 120, 160, 1, oracle.SPLIT, 8),
           _scene(1, 5, 9, 150, 200, 2, oracle.SPLIT, 0),
           _scene(2, 21, 13, 96, 128, 1, oracle.SQUARE, 4, fp8=True)]
    for d in out:
        om = oracle_mesh(d["sc"].vertices, d["sc"].faces, d["s"], d["scheme"])
        _, l_o = om.raster_frames(d["cams"], d["H"], d["W"])
        F = len(d["cams"])
        idx = np.arange(F) % d["pool"] if d["pool"] else np.arange(F)
        if d["fp8"]:
            A, Ws = oracle.fuse(om.n_texels, 13, l_o, d["q"].numpy()[idx], d["valid"].numpy()[idx],
                                scale=d["scale"].numpy()[idx])
        else:
            A, Ws = oracle.fuse(om.n_texels, 13, l_o, d["probs"].numpy()[idx], d["valid"].numpy()[idx])
        P, lab = oracle.finalize(A, Ws)
        d.update(om=om, l_o=l_o, P_o=P, lab_o=lab, valid_exp=d["valid"].numpy()[idx])
    return out


def _jobs(scs, batches=(8, 4, 16), tunings=None):
    jobs, meshes = [], []
    for i, d in enumerate(scs):
        m = sf.Mesh(to_dev(d["sc"].vertices, torch.float32), to_dev(d["sc"].faces, torch.int32), n_classes=13,
                    s=d["s"], scheme=d["scheme"])
        if tunings:
            m.set_tuning(**tunings[i])
        cams = to_dev(d["cams"], torch.float32)
        if d["fp8"]:
            probs, scale = d["q"].cuda().to(memory_format=torch.channels_last), d["scale"].cuda()
        else:
            probs, scale = d["probs"].cuda().to(memory_format=torch.channels_last), None
        jobs.append(m.job(cams, probs, scale=scale, valid=d["valid"].cuda(), pool=d["pool"], batch=batches[i],
                          tex_dtype=torch.float32, images=True))
        meshes.append(m)
    return jobs, meshes


def _check(jobs, scs, tag):
    torch.cuda.synchronize()
    for j, d in zip(jobs, scs):
        assert np.array_equal(j.l.cpu().numpy(), d["l_o"]), f"{tag}: texel rows differ"
        compare_normalized(j.tex.cpu().numpy(), d["P_o"])
        compare_labels(j.labels.cpu().numpy(), d["P_o"], d["lab_o"])
        lab = j.labels.cpu().numpy()
        assert np.array_equal(j.images.cpu().numpy(), oracle.render(d["l_o"], lab, d["valid_exp"])), \
            f"{tag}: rendered label images differ"


def test_fuse_batch_matches_oracle(scenes):
    jobs, _ = _jobs(scenes)
    sf.fuse_batch(jobs)
    _check(jobs, scenes, "eager batch")


def test_tunings_do_not_change_results(scenes):
    d = scenes[0]
    for tile, unroll, small, gw in ((16, 4, 12, 8), (16, 8, 1, 1), (32, 4, 96, 32), (32, 8, 48, 512)):
        t = {"tile": tile, "gather_unroll": unroll, "small_px": small, "gather_waves": gw}
        jobs, meshes = _jobs(scenes[:1], tunings=[t])
        assert meshes[0].get_tuning() == dict(t, learned_in_gather=0)
        sf.fuse_batch(jobs)
        _check(jobs, scenes[:1], f"tile {tile} unroll {unroll}")
        r = meshes[0].rasterize(to_dev(d["cams"], torch.float32), d["H"], d["W"])
        assert np.array_equal(r["l"].cpu().numpy(), d["l_o"])
    # gathers on the caller's stream (no overlap between batches)
    jobs, meshes2 = _jobs(scenes[:1])
    meshes2[0].set_overlap(False)
    sf.fuse_batch(jobs)
    _check(jobs, scenes[:1], "no overlap")
    # FP8 channels-last input (scene 2) through the gather's 4-deep unroll and the smallest grid
    for unroll, gw in ((4, 1), (4, 8), (8, 32)):
        t = {"tile": 16, "gather_unroll": unroll, "small_px": 24, "gather_waves": gw}
        jobs, _ = _jobs(scenes[2:], batches=(5,), tunings=[t])
        sf.fuse_batch(jobs)
        _check(jobs, scenes[2:], f"FP8 unroll {unroll} waves {gw}")
    with pytest.raises(sf.SemfuseError):
        meshes[0].set_tuning(24, 8)
    with pytest.raises(sf.SemfuseError):
        meshes[0].set_tuning(32, 8, 0)
    with pytest.raises(sf.SemfuseError):
        meshes[0].set_tuning(32, 8, 48, 1025)


def test_graph_replays_match_oracle(scenes):
    """Capture all three scenes' fusions as one graph; replay three times with
    eager library work in between; every replay is checked."""
    jobs, meshes = _jobs(scenes)
    g = sf.Graph(jobs)
    eager_jobs, _ = _jobs(scenes, batches=(3, 7, 5))
    for rep in range(3):
        for j in jobs:                      # poison the outputs
            j.labels.fill_(77)
            j.tex.fill_(-1.0)
            j.images.fill_(77)
        g.launch()
        torch.cuda.synchronize()
        _check(jobs, scenes, f"replay {rep}")
        sf.fuse_batch(eager_jobs)           # eager work between replays
        torch.cuda.synchronize()
        _check(eager_jobs, scenes, f"eager after replay {rep}")


def test_autotuner_picks_and_caches(scenes, tmp_path):
    d = scenes[0]
    m = sf.Mesh(to_dev(d["sc"].vertices, torch.float32), to_dev(d["sc"].faces, torch.int32), n_classes=13, s=1,
                scheme=oracle.SPLIT)
    cams = to_dev(d["cams"][:8], torch.float32)
    probs = d["probs"].cuda().to(memory_format=torch.channels_last)
    path = str(tmp_path / "tune.json")
    r1 = tune.autotune(m, cams, probs, valid=d["valid"].cuda(), probe_frames=8, cache_path=path, log=say)
    assert not r1["cached"] and r1["n_candidates"] >= 6
    got = m.get_tuning()
    assert {k: got[k] for k in ("tile", "gather_unroll", "small_px", "gather_waves")} == \
        {k: r1[k] for k in ("tile", "gather_unroll", "small_px", "gather_waves")}
    with open(path) as fh:
        table = json.load(fh)
    assert len(table) == 1
    r2 = tune.autotune(m, cams, probs, valid=d["valid"].cuda(), probe_frames=8, cache_path=path)
    knobs = ("tile", "gather_unroll", "small_px", "gather_waves", "batch", "scatter_mode")
    assert r2["cached"] and {k: r2[k] for k in knobs} == {k: r1[k] for k in knobs}
    # the accumulator is left clear
    assert float(m.accum.abs().max()) == 0.0


def test_batch_errors_are_reported(scenes):
    jobs, _ = _jobs(scenes[:1])
    bad = jobs[0]
    bad.st.batch = 0
    with pytest.raises(sf.SemfuseError):
        sf.fuse_batch([bad], ws=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
