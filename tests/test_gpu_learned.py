"""Learned per-observation weight on the GPU against the binary64 oracle:
network forward, gradients, Adam, per-observation features, fusion with the
weight inferred inside the fusion pass, and training + held-out gain.  All
calls go through the C-ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
from paper_2111_11103_amd import learned as LR
from paper_2111_11103_amd import scenes as S
from paper_2111_11103_amd import semfuse as sf
from tests.gpu_cases import gpu_mesh, oracle_mesh, say, to_dev

pytestmark = pytest.mark.gpu


def _phi(n, seed):
    g = np.random.default_rng(seed)
    x = g.random((n, 8)).astype(np.float32)
    x[:, 6] *= 2.0
    return x


def _params(seed, b1=0.1):
    p = sf.init_params(seed).numpy().copy()
    # a positive first-layer bias keeps both ReLU branches populated
    p[8 * 64:8 * 64 + 64] = b1
    return p


def test_mlp_forward_matches_oracle():
    """Same inputs and weights.  The kernel sums exact bfloat16 products in
    binary32 (8 or 64 terms: relative error <= 64 * 2^-24 of the absolute
    sum), so the output differs from the binary64 oracle by ~1e-6; where that
    difference moves a hidden unit across a bfloat16 rounding boundary the
    unit changes by one bfloat16 ulp (2^-8 relative), bounded here by 2e-3 on
    the weight."""
    say("[case] mlp forward, n = 5037 (ragged)")
    for seed in (1, 2):
        p = _params(seed)
        phi = _phi(5037, seed)
        mlp = sf.WeightMLP("cuda", torch.from_numpy(p))
        w = mlp.forward(to_dev(phi)).cpu().numpy().astype(np.float64)
        ref = omlp.forward(p, phi, round_mode=1)
        d = np.abs(w - ref)
        say(f"  seed {seed}: w in [{ref.min():.3f}, {ref.max():.3f}]  max |dw| {d.max():.2e}  "
            f"99th pct {np.quantile(d, 0.99):.2e}")
        assert d.max() <= 2e-3
        assert np.quantile(d, 0.99) <= 1e-5
    # empty input is a no-op
    assert mlp.forward(torch.empty((0, 8), device="cuda")).numel() == 0


def test_mlp_gradients_match_oracle():
    """Straight-through gradients of the mean BCE: binary32 kernel vs binary64
    oracle on identical weights and batches, within 2e-2 of the largest
    component (bfloat16 level)."""
    say("[case] mlp gradients, n = 3000 (ragged)")
    for seed in (3, 4):
        p = _params(seed)
        phi = _phi(3000, seed + 10)
        y = (np.random.default_rng(seed).random(3000) < 0.6).astype(np.float32)
        mlp = sf.WeightMLP("cuda", torch.from_numpy(p))
        loss, g = mlp.loss_grad(to_dev(phi), to_dev(y))
        g = g.cpu().numpy().astype(np.float64)
        loss = float(loss.item())
        l_ref, g_ref = omlp.loss_grad(p, phi, y, round_mode=1)
        scale = np.abs(g_ref).max()
        err = np.abs(g - g_ref)
        say(f"  seed {seed}: loss {loss:.6f} vs {l_ref:.6f}  max |dg| / max |g| = {err.max() / scale:.2e}")
        assert abs(loss - l_ref) <= 1e-4 * max(1.0, abs(l_ref))
        assert err.max() <= 2e-2 * scale
        # blockwise: every parameter group is right on its own scale
        for lo, hi in ((0, 512), (512, 576), (576, 4672), (4672, 4736), (4736, 4800), (4800, 4801)):
            sc = max(np.abs(g_ref[lo:hi]).max(), 1e-3 * scale)
            assert np.abs(g[lo:hi] - g_ref[lo:hi]).max() <= 2e-2 * sc, (lo, hi)


def test_mlp_gradient_of_empty_batch_is_zero():
    mlp = sf.WeightMLP("cuda", torch.from_numpy(_params(5)))
    loss, g = mlp.loss_grad(torch.empty((0, 8), device="cuda"), torch.empty(0, device="cuda"))
    assert float(g.abs().max()) == 0.0 and float(loss.item()) == 0.0


def test_adam_matches_oracle():
    n = sf.mlp_sizes()[0]
    p0 = _params(6)
    mlp = sf.WeightMLP("cuda", torch.from_numpy(p0))
    rng = np.random.default_rng(6)
    p_ref = p0.copy()
    m = np.zeros(n)
    v = np.zeros(n)
    for t in range(1, 4):
        g = rng.normal(0, 1, n).astype(np.float32)
        mlp.adam(to_dev(g), lr=1e-3)
        p_ref = omlp.adam(p_ref, m, v, g.astype(np.float64), lr=1e-3, t=t)
    got = mlp.params.cpu().numpy()
    # binary32 vs binary64 arithmetic: about ten roundings (unit 2^-24) per
    # step over three steps, relative to the parameter and to the distance it
    # moved (at most lr per step)
    assert np.all(np.abs(got.astype(np.float64) - p_ref) <= 2e-6 * (np.abs(p_ref) + 3 * 1e-3))
    # the packed bfloat16 weights are the round-to-nearest-even of the masters
    mlp2 = sf.WeightMLP("cuda", torch.from_numpy(p_ref))
    w = mlp2.forward(to_dev(_phi(64, 0))).cpu().numpy()
    assert np.allclose(w, omlp.forward(p_ref, _phi(64, 0)), atol=2e-3)


@pytest.fixture(scope="module")
def scene():
    say("[case] learned features / fusion on config-1 (structured noise), 6 frames")
    w = S.config1(device="cpu", structured=True, n_frames=6)
    sc = w.scene
    om = oracle_mesh(sc.vertices, sc.faces, 1, oracle.SPLIT)
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    A, Ws = oracle.fuse(om.n_texels, 13, l_o, w.probs.numpy(), w.valid.numpy())
    _, lab = oracle.finalize(A, Ws)
    return w, om, l_o, A, lab


def _oracle_features(w, om, lab, probs=None):
    probs = w.probs.numpy() if probs is None else probs
    HW = w.H * w.W
    phis, tgts, pixs = [], [], []
    for f in range(len(w.cams)):
        phi, tgt, pix = omlp.frame_features(om, w.cams[f], w.H, w.W, probs[f], w.valid.numpy()[f], lab)
        phis.append(phi)
        tgts.append(tgt)
        pixs.append(pix.astype(np.int64) + f * HW)
    return np.concatenate(phis), np.concatenate(tgts), np.concatenate(pixs)


@pytest.mark.parametrize("fp8", [False, True])
def test_features_match_oracle(scene, fp8):
    """Same observation set and targets (exact); features within binary32
    rounding of the binary64 definitions (the viewing-angle cosine is built
    from binary32 camera-space vertices on the GPU: 1e-4)."""
    w, om, l_o, _, lab = scene
    sc = w.scene
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, 13)
    if fp8:
        q, scale = S.quantize_fp8(w.probs)
        deq = np.vectorize(oracle.e4m3_decode)(np.arange(256)).astype(np.float32)[q.numpy()]
        probs_o = (deq * scale.numpy()[:, None]).astype(np.float32)
        phi, tgt, pix = gm.extract_features(to_dev(w.cams, torch.float32), q.cuda(), scale=scale.cuda(),
                                            valid=w.valid.cuda(), labels=to_dev(lab))
    else:
        probs_o = None
        phi, tgt, pix = gm.extract_features(to_dev(w.cams, torch.float32), w.probs.cuda(), valid=w.valid.cuda(),
                                            labels=to_dev(lab))
    torch.cuda.synchronize()
    order = torch.argsort(pix.long()).cpu().numpy()
    phi, tgt, pix = phi.cpu().numpy()[order], tgt.cpu().numpy()[order], pix.cpu().numpy()[order]
    phi_o, tgt_o, pix_o = _oracle_features(w, om, lab, probs_o)
    assert np.array_equal(pix.astype(np.int64), pix_o)
    assert np.array_equal(tgt, tgt_o)
    d = np.abs(phi.astype(np.float64) - phi_o)
    say(f"  fp8={fp8}: {len(pix)} observations, max |dphi| per feature " + " ".join(f"{x:.1e}" for x in d.max(0)))
    assert d[:, 0].max() <= 1e-4
    assert d[:, 1:].max() <= 2e-5


@pytest.mark.parametrize("mode", [sf.SCATTER_ATOMIC, sf.SCATTER_SORTED])
def test_learned_fusion_matches_oracle(scene, mode):
    """Fusion with the weight inferred inside the fusion pass against the
    oracle chain (binary64 features -> binary64 network -> binary64 fusion).
    A weight may differ by up to delta = 5e-3 where a feature's bfloat16
    rounding falls differently (features agree to 1e-4); so every element is
    bounded by 1e-5 |A| + delta * (unweighted sum), and most texels, which
    see no such observation, agree to 1e-5."""
    w, om, l_o, A_plain, lab = scene
    sc = w.scene
    p = _params(7)
    phi_o, _, pix_o = _oracle_features(w, om, lab)
    wts = omlp.forward(p, phi_o).astype(np.float32)
    wpix = np.zeros(l_o.shape, np.float32).reshape(-1)
    wpix[pix_o] = wts
    A_o, W_o = oracle.fuse(om.n_texels, 13, l_o, w.probs.numpy(), w.valid.numpy(), weighting=oracle.W_GIVEN,
                           wpix=wpix.reshape(l_o.shape))
    probs = w.probs.cuda() if mode == sf.SCATTER_ATOMIC else w.probs.permute(0, 2, 3, 1).contiguous().cuda().permute(
        0, 3, 1, 2)
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, 13)
    mlp = sf.WeightMLP("cuda", torch.from_numpy(p))
    with pytest.raises(sf.SemfuseError):
        gm.fuse_frames(to_dev(w.cams, torch.float32), probs, valid=w.valid.cuda(), weighting=sf.W_LEARNED)
    gm.bind_mlp(mlp)
    gm.fuse_frames(to_dev(w.cams, torch.float32), probs, valid=w.valid.cuda(), weighting=sf.W_LEARNED,
                   scatter_mode=mode, batch=4)
    A = gm.accum.cpu().numpy().astype(np.float64)
    Wg = gm.wsum.cpu().numpy().astype(np.float64)
    delta = 5e-3
    err = np.abs(A - A_o)
    assert np.all(err <= 1e-5 * np.abs(A_o) + delta * A_plain + 1e-30)
    rel_row = (err / np.maximum(np.abs(A_o), 1e-30)).max(1)
    seen = W_o > 0
    frac = float((rel_row[seen] <= 1e-5).mean())
    say(f"  mode {mode}: texels within 1e-5: {frac:.3f}; max row rel {rel_row[seen].max():.2e}; "
        f"weights in [{wts.min():.3f}, {wts.max():.3f}]")
    assert frac >= 0.99
    n_obs = np.bincount(l_o[(l_o >= 0) & (w.valid.numpy() != 0)], minlength=om.n_texels)
    assert np.all(np.abs(Wg - W_o) <= 1e-5 * W_o + delta * n_obs)
    # labels: equal wherever the oracle's margin exceeds the weight tolerance
    P_o, lab_o = oracle.finalize(A_o, W_o)
    tex, lab_g = gm.finalize()
    lab_g = lab_g.cpu().numpy()
    srt = np.sort(P_o, 1)
    margin = srt[:, -1] - srt[:, -2]
    tol = 2 * delta * A_plain.sum(1) / np.maximum(A_o.sum(1), 1e-30) + 1e-5
    sure = seen & (margin > tol)
    assert np.array_equal(lab_g[sure], lab_o[sure])
    assert float((lab_g[seen] == lab_o[seen]).mean()) >= 0.99


@pytest.mark.parametrize("layout", ["nhwc", "staged", "fp8"])
def test_learned_fusion_on_grouped_gather(scene, layout):
    """c = 16 (classes in 4-class chunks), learned_in_gather = 1: the
    texel-sorted gather evaluates the network for every observation itself (features from the observation's
    own class vector, n from its per-row frame counters, geometry from the
    resolve's per-set copy) for channels-last input, planar input staged as
    rows and channels-last E4M3 input with its per-pixel scale; batches of 2
    and 4 frames (3 and 2 batches, both geometry sets in use).  Same bound as
    the fusion test above."""
    w, om, l_o, _, lab = scene
    sc = w.scene
    c = 16
    g = torch.Generator().manual_seed(77)
    probs = torch.softmax(2.0 * torch.randn((len(w.cams), c, w.H, w.W), generator=g), 1)
    scale = None
    if layout == "fp8":
        q, scale = S.quantize_fp8(probs)
        deq = np.vectorize(oracle.e4m3_decode)(np.arange(256)).astype(np.float32)[q.numpy()]
        probs_o = (deq * scale.numpy()[:, None]).astype(np.float32)
        x = q.permute(0, 2, 3, 1).contiguous().cuda().permute(0, 3, 1, 2)
        scale = scale.cuda()
    else:
        probs_o = probs.numpy()
        x = probs.to(memory_format=torch.channels_last).cuda() if layout == "nhwc" else probs.cuda()
    p = _params(7)
    phi_o, _, pix_o = _oracle_features(w, om, lab, probs=probs_o)
    wts = omlp.forward(p, phi_o).astype(np.float32)
    wpix = np.zeros(l_o.shape, np.float32).reshape(-1)
    wpix[pix_o] = wts
    A_o, W_o = oracle.fuse(om.n_texels, c, l_o, probs_o, w.valid.numpy(), weighting=oracle.W_GIVEN,
                           wpix=wpix.reshape(l_o.shape))
    A_plain, _ = oracle.fuse(om.n_texels, c, l_o, probs_o, w.valid.numpy())
    mode = sf.SCATTER_STAGED if layout == "staged" else sf.SCATTER_SORTED
    mlp = sf.WeightMLP("cuda", torch.from_numpy(p))
    for batch in (2, 4):
        say(f"  learned weight, {layout}, batch {batch}")
        gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, c)
        gm.bind_mlp(mlp)
        gm.set_tuning(learned_in_gather=1)
        gm.fuse_frames(to_dev(w.cams, torch.float32), x, scale=scale, valid=w.valid.cuda(), weighting=sf.W_LEARNED,
                       scatter_mode=mode, batch=batch)
        A = gm.accum.cpu().numpy().astype(np.float64)
        delta = 5e-3
        err = np.abs(A - A_o)
        assert np.all(err <= 1e-5 * np.abs(A_o) + delta * A_plain + 1e-30)
        rel_row = (err / np.maximum(np.abs(A_o), 1e-30)).max(1)
        seen = W_o > 0
        frac = float((rel_row[seen] <= 1e-5).mean())
        say(f"    texels within 1e-5: {frac:.4f}")
        assert frac >= 0.99
        # the separate inference pass computes the same weights; the sums
        # differ only in the order of the observations within a row
        gm.set_tuning(learned_in_gather=0)
        gm.reset()
        gm.fuse_frames(to_dev(w.cams, torch.float32), x, scale=scale, valid=w.valid.cuda(), weighting=sf.W_LEARNED,
                       scatter_mode=mode, batch=batch)
        A0 = gm.accum.cpu().numpy().astype(np.float64)
        d01 = np.abs(A0 - A) / np.maximum(np.abs(A), 1e-30)
        say(f"    separate pass vs in the gather: max rel {d01.max():.2e}")
        assert np.all(np.abs(A0 - A) <= 1e-5 * np.abs(A) + 1e-30)


def test_learned_in_gather_at_forty_classes():
    """Both sites of the network at c = 40 (ten active lanes of a row
    group), in batches of 64 (per-frame counters for 64 frames) and of 32
    (three batches: a buffer set reused), SPLIT s = 3 texels: inside the
    gather, and in its own pass; fusion against the oracle chain, same
    bound as above."""
    say("[case] learned weight at c = 40, 90 frames of 160x120, batches 64 and 32, both sites")
    w = S.config1(device="cpu", structured=True, n_frames=90)
    sc = w.scene
    om = oracle_mesh(sc.vertices, sc.faces, 3, oracle.SPLIT)
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    c = 40
    g = torch.Generator().manual_seed(5)
    probs = torch.softmax(2.5 * torch.randn((len(w.cams), c, w.H, w.W), generator=g), 1)
    A_p, W_p = oracle.fuse(om.n_texels, c, l_o, probs.numpy(), w.valid.numpy())
    _, lab = oracle.finalize(A_p, W_p)
    p = _params(11)
    phi_o, _, pix_o = _oracle_features(w, om, lab, probs=probs.numpy())
    wts = omlp.forward(p, phi_o).astype(np.float32)
    wpix = np.zeros(l_o.shape, np.float32).reshape(-1)
    wpix[pix_o] = wts
    A_o, W_o = oracle.fuse(om.n_texels, c, l_o, probs.numpy(), w.valid.numpy(), weighting=oracle.W_GIVEN,
                           wpix=wpix.reshape(l_o.shape))
    gm = gpu_mesh((sc.vertices, sc.faces), 3, oracle.SPLIT, c)
    gm.bind_mlp(sf.WeightMLP("cuda", torch.from_numpy(p)))
    x = probs.to(memory_format=torch.channels_last).cuda()
    # inside the gather, then the separate pass
    for site, batch in ((1, 64), (1, 32), (0, 64), (0, 32)):
        gm.set_tuning(32, 8, 96, 8, learned_in_gather=site)
        gm.reset()
        gm.fuse_frames(to_dev(w.cams, torch.float32), x, valid=w.valid.cuda(), weighting=sf.W_LEARNED,
                       scatter_mode=sf.SCATTER_SORTED, batch=batch)
        A = gm.accum.cpu().numpy().astype(np.float64)
        delta = 5e-3
        err = np.abs(A - A_o)
        assert np.all(err <= 1e-5 * np.abs(A_o) + delta * A_p + 1e-30)
        rel_row = (err / np.maximum(np.abs(A_o), 1e-30)).max(1)
        seen = W_o > 0
        frac = float((rel_row[seen] <= 1e-5).mean())
        say(f"  site {site}, batch {batch}: texels within 1e-5: {frac:.4f} of {int(seen.sum())}")
        assert frac >= 0.99


@pytest.mark.parametrize("dtype,c", [("f32", 40), ("fp8", 20), ("f32", 4), ("f32", 64)])
def test_learned_sites_on_ragged_frames(dtype, c):
    """Both sites of the network for pixel-dense channels-last input.  In its
    own pass the class vectors are copied to LDS a wave (64 pixels) at a
    time: 157x113 frames end in a partial wave of 13 pixels (for that pass
    the E4M3 input, c = 20, has its frames padded to a 16-byte stride, so
    that wave's bytes end in a 4-byte word; the gather takes dense frames
    only and gets them unpadded).  Inside the gather four
    lanes read a vector, lane j its chunks j, j + 4, ...: c = 4 (one chunk),
    20 (lane 0 two chunks, the others one), 40 (up to three), 64 (four each).
    10 % of the pixels invalid.  Fusion against the oracle chain, same bound
    as above."""
    say(f"[case] learned weight, both sites, {dtype} c = {c}, 6 frames of 157x113 (ragged last wave)")
    w = S.config1(device="cpu", structured=True, n_frames=6, H=113, W=157)
    g = torch.Generator().manual_seed(31)
    valid = w.valid.clone()
    valid[torch.rand(valid.shape, generator=g) < 0.1] = 0
    w.valid = valid
    sc = w.scene
    om = oracle_mesh(sc.vertices, sc.faces, 1, oracle.SPLIT)
    _, l_o = om.raster_frames(w.cams, w.H, w.W)
    probs = torch.softmax(2.0 * torch.randn((len(w.cams), c, w.H, w.W), generator=g), 1)
    scale = None
    if dtype == "fp8":
        q, scale = S.quantize_fp8(probs)
        deq = np.vectorize(oracle.e4m3_decode)(np.arange(256)).astype(np.float32)[q.numpy()]
        probs_o = (deq * scale.numpy()[:, None]).astype(np.float32)
        F, n = len(w.cams), w.H * w.W * c
        fstride = (n + 15) // 16 * 16
        assert fstride != n and (13 * c) % 16 != 0
        buf = torch.zeros((F, fstride), dtype=torch.uint8)
        buf[:, :n] = q.permute(0, 2, 3, 1).reshape(F, n)
        xs = {0: buf.cuda().as_strided((F, c, w.H, w.W), (fstride, 1, w.W * c, c)),
              1: q.permute(0, 2, 3, 1).contiguous().cuda().permute(0, 3, 1, 2)}
        scale = scale.cuda()
    else:
        probs_o = probs.numpy()
        x = probs.to(memory_format=torch.channels_last).cuda()
        xs = {0: x, 1: x}
    A_p, W_p = oracle.fuse(om.n_texels, c, l_o, probs_o, w.valid.numpy())
    _, lab = oracle.finalize(A_p, W_p)
    p = _params(13)
    phi_o, _, pix_o = _oracle_features(w, om, lab, probs=probs_o)
    wts = omlp.forward(p, phi_o).astype(np.float32)
    wpix = np.zeros(l_o.shape, np.float32).reshape(-1)
    wpix[pix_o] = wts
    A_o, W_o = oracle.fuse(om.n_texels, c, l_o, probs_o, w.valid.numpy(), weighting=oracle.W_GIVEN,
                           wpix=wpix.reshape(l_o.shape))
    gm = gpu_mesh((sc.vertices, sc.faces), 1, oracle.SPLIT, c)
    gm.bind_mlp(sf.WeightMLP("cuda", torch.from_numpy(p)))
    for site, batch in ((0, 2), (0, 6), (1, 2), (1, 6)):
        gm.set_tuning(learned_in_gather=site)
        gm.reset()
        gm.fuse_frames(to_dev(w.cams, torch.float32), xs[site], scale=scale, valid=w.valid.cuda(),
                       weighting=sf.W_LEARNED, scatter_mode=sf.SCATTER_SORTED, batch=batch)
        A = gm.accum.cpu().numpy().astype(np.float64)
        delta = 5e-3
        err = np.abs(A - A_o)
        assert np.all(err <= 1e-5 * np.abs(A_o) + delta * A_p + 1e-30)
        rel_row = (err / np.maximum(np.abs(A_o), 1e-30)).max(1)
        seen = W_o > 0
        frac = float((rel_row[seen] <= 1e-5).mean())
        say(f"  site {site}, batch {batch}: texels within 1e-5: {frac:.4f} of {int(seen.sum())}")
        assert frac >= 0.99


def test_training_and_heldout_gain():
    """Train on 50 seeded scenes (seeds 100-149, view-dependent noise) with the
    project's kernels, then fuse 10 held-out scenes (seeds 200-209) with the
    input argmax, w^(P), w^(I), the learned weight, and the judged form (the
    learned weight where plain fusion's held-out-frame judge keeps it, w = 1
    where it falls back).  Pinned: the loss falls below the constant
    predictor's; plain fusion beats the input argmax; the judged form's
    held-out agreement is never below plain fusion's, and where it falls back
    its accuracy is plain fusion's exactly.  The gain itself is reported, not
    pinned (parity unpinned: no paper number exists for it)."""
    say("[case] learned weight: training on seeds 100-149, evaluation on 200-209")
    phi, tgt = LR.training_set(range(100, 150), device="cuda", structured=True, log=say)
    pos = float(tgt.mean())
    h_const = -(pos * math.log(pos) + (1 - pos) * math.log(1 - pos))
    mlp = sf.WeightMLP("cuda", seed=0)
    l0 = LR.full_loss(mlp, phi, tgt)
    LR.train(mlp, phi, tgt, steps=1500, batch=32768, lr=2e-3, log=say, log_every=300)
    l1 = LR.full_loss(mlp, phi, tgt)
    say(f"  full-set loss {l0:.4f} -> {l1:.4f}   (constant predictor {h_const:.4f})")
    assert l1 < l0 and l1 < 0.97 * h_const
    rows = []
    for structured in (True, False):
        for step in (1, 4):
            acc = {"input": [], "pixel": [], "image": [], "learned": [], "judged": []}
            kept = 0
            for sd in range(200, 210):
                w = LR.subsample(S.config1(device="cuda", seed=sd, structured=structured), step)
                r = LR.evaluate(w, mlp)
                mesh = LR.scene_mesh(w, "cuda")
                j = LR.judge(mesh, torch.as_tensor(w.cams, dtype=torch.float32, device="cuda"), w.probs.cuda(), mlp,
                             valid=w.valid.cuda(), holdout_every=4 if step == 1 else 2)
                assert max(j["agreement_learned"], j["agreement_plain"]) >= j["agreement_plain"]
                kept += j["choice"] == sf.W_LEARNED
                r["judged"] = r["learned"] if j["choice"] == sf.W_LEARNED else r["pixel"]
                for k in acc:
                    acc[k].append(r[k])
            m = {k: float(np.mean(v)) for k, v in acc.items()}
            rows.append((structured, step, m))
            say(f"  held-out {'structured' if structured else 'plain     '} noise, {20 // step:2d} frames: "
                f"input {m['input']:.4f}  w^P {m['pixel']:.4f}  w^I {m['image']:.4f}  learned {m['learned']:.4f}  "
                f"judged {m['judged']:.4f} (learned kept on {kept}/10)  "
                f"gain vs w^P: learned {m['learned'] - m['pixel']:+.4f}, judged {m['judged'] - m['pixel']:+.4f}")
    for structured, step, m in rows:
        assert m["pixel"] > m["input"]


def test_judge_falls_back_on_a_harmful_weight():
    """A network that trusts uncertain observations and all but ignores
    confident ones (w = sigmoid(48 relu(0.5 - top-1) - 6)) makes the fused
    labels worse on every scene; plain fusion's held-out-frame judge must
    reject it on every scene, so the judged form is plain fusion."""
    NI, NH = 8, 64
    o_b1 = NH * NI
    o_w2 = o_b1 + NH
    o_b2 = o_w2 + NH * NH
    o_w3 = o_b2 + NH
    o_b3 = o_w3 + NH
    harm = np.zeros(omlp.nparam(), np.float32)
    harm[0 * NI + 3] = -1.0            # h1_0 = relu(0.5 - top1)
    harm[o_b1 + 0] = 0.5
    harm[o_w2 + 0 * NH + 0] = 1.0      # h2_0 = h1_0
    harm[o_w3 + 0] = 48.0              # w = sigmoid(48 h2_0 - 6): ~1 where top1 < 0.37, 0.0025 where top1 >= 0.5
    harm[o_b3] = -6.0
    bad = sf.WeightMLP("cuda", torch.from_numpy(harm))
    falls = 0
    for sd in range(200, 206):
        w = S.config1(device="cuda", seed=sd, structured=True)
        mesh = LR.scene_mesh(w, "cuda")
        j = LR.judge(mesh, torch.as_tensor(w.cams, dtype=torch.float32, device="cuda"), w.probs.cuda(), bad,
                     valid=w.valid.cuda(), holdout_every=4)
        r = LR.evaluate(w, bad)
        say(f"  seed {sd}: agreement plain {j['agreement_plain']:.4f} harmful {j['agreement_learned']:.4f}; "
            f"accuracy plain {r['pixel']:.4f} harmful {r['learned']:.4f}")
        assert r["learned"] < r["pixel"]
        falls += j["choice"] == sf.W_PIXEL
    assert falls == 6
