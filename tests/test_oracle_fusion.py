"""Pins of the oracle's fusion (Section 3.2.1 eqs. maxsum/mul/sum, Section
3.2.2 eqs. w-maxsum/w-mul/w-sum and the weights w^(P), w^(I), Section 3.3.2
eq. texel-in-array), normalisation, argmax and render-back.  CPU only."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(1234)


def _frames(F, H, W, n_tex, invalid=0.0, rng=RNG):
    l = rng.integers(-1, n_tex, (F, H, W)).astype(np.int32)
    valid = (rng.random((F, H, W)) >= invalid).astype(np.uint8)
    return l, valid


def _probs_from_rows(q, l, c, rng=RNG):
    """p_k = q[l_k] for covered pixels, a random distribution elsewhere; NCHW."""
    F, H, W = l.shape
    noise = rng.dirichlet(np.ones(c), size=(F, H, W))
    p = np.where((l >= 0)[..., None], q[np.maximum(l, 0)], noise)
    return np.ascontiguousarray(p.transpose(0, 3, 1, 2)).astype(np.float32)


def _exact_simplex(size, c, rng=RNG):
    """Random distributions with dyadic entries that sum to exactly 1 in binary32."""
    cuts = np.sort(rng.integers(0, 4097, size=tuple(size) + (c - 1,)), axis=-1)
    edges = np.concatenate([np.zeros(tuple(size) + (1,), np.int64), cuts,
                            np.full(tuple(size) + (1,), 4096, np.int64)], -1)
    return (np.diff(edges, axis=-1) / 4096.0).astype(np.float32)


def test_unanimous_frames_are_a_fixed_point():
    """Every observation of texel x equals q_x  =>  P_x = q_x (any weighting,
    aggregator sum or maxsum-free), and fuse -> render -> fuse is unchanged."""
    c, n = 7, 50
    q = RNG.dirichlet(np.ones(c), size=n).astype(np.float32).astype(np.float64)
    l, valid = _frames(6, 9, 11, n, invalid=0.2)
    p = _probs_from_rows(q, l, c)
    for wt in (oracle.W_PIXEL, oracle.W_IMAGE):
        A, Ws = oracle.fuse(n, c, l, p, valid, weighting=wt)
        P, lab = oracle.finalize(A, Ws)
        seen = np.zeros(n, bool)
        seen[l[(l >= 0) & (valid > 0)]] = True
        qn = q / q.sum(1, keepdims=True)   # q is binary32-rounded: its norm is the fixed point
        assert np.allclose(P[seen], qn[seen], rtol=1e-12, atol=0)
        assert (P[~seen] == 0).all() and (lab[~seen] == 255).all()
        assert np.array_equal(lab[seen], q[seen].argmax(1))
        # render the fused labels back as one-hot distributions and fuse again
        out = oracle.render(l, lab, valid)
        assert ((out == 255) == ((l < 0) | (valid == 0))).all()
        onehot = np.eye(c, dtype=np.float32)[np.minimum(out, c - 1)].transpose(0, 3, 1, 2)
        A2, W2 = oracle.fuse(n, c, l, np.ascontiguousarray(onehot), valid, weighting=wt)
        _, lab2 = oracle.finalize(A2, W2)
        assert np.array_equal(lab2, lab)


def test_single_frame_reproduces_input_argmax():
    """One frame whose pixels on the same texel agree: rendering the fused
    texture gives every visible valid pixel its own argmax."""
    c, n = 5, 30
    q = RNG.dirichlet(np.ones(c) * 0.5, size=n)
    l, valid = _frames(1, 20, 20, n, invalid=0.1)
    p = _probs_from_rows(q, l, c)
    A, Ws = oracle.fuse(n, c, l, p, valid)
    _, lab = oracle.finalize(A, Ws)
    out = oracle.render(l, lab, valid)
    vis = (l >= 0) & (valid > 0)
    assert np.array_equal(out[vis], p.argmax(1)[vis])
    assert (out[~vis] == 255).all()


def test_weighting_closed_forms():
    """w^(P): P_x = mean of p_k over K_x (Sigma_j p_kj = 1 makes norm the mean).
    w^(I): P_x = mean over frames i seeing x of the per-frame mean over
    K_i ∩ K_x (Section 3.2.2)."""
    c, n, F, H, W = 4, 12, 5, 8, 10
    l, valid = _frames(F, H, W, n, invalid=0.15)
    p = _exact_simplex((F, H, W), c)
    pn = np.ascontiguousarray(p.transpose(0, 3, 1, 2))
    m = (l >= 0) & (valid > 0)
    pd = p.astype(np.float64)
    ref_P = np.zeros((n, c))
    ref_I = np.zeros((n, c))
    for x in range(n):
        sel = m & (l == x)
        if sel.any():
            ref_P[x] = pd[sel].mean(0)
            per = [pd[f][sel[f]].mean(0) for f in range(F) if sel[f].any()]
            ref_I[x] = np.mean(per, 0)
    A, Ws = oracle.fuse(n, c, l, pn, valid, weighting=oracle.W_PIXEL)
    P, _ = oracle.finalize(A, Ws)
    assert np.allclose(P, ref_P, rtol=1e-12, atol=1e-15)
    A, Ws = oracle.fuse(n, c, l, pn, valid, weighting=oracle.W_IMAGE)
    P, _ = oracle.finalize(A, Ws)
    assert np.allclose(P, ref_I, rtol=1e-12, atol=1e-15)
    # the total weight per texel: pixel count (w^(P)), frame count (w^(I))
    _, Ws_p = oracle.fuse(n, c, l, pn, valid, weighting=oracle.W_PIXEL)
    assert np.array_equal(Ws_p, np.bincount(l[m], minlength=n).astype(np.float64))
    frames_seen = np.array([sum((m[f] & (l[f] == x)).any() for f in range(F)) for x in range(n)], np.float64)
    assert np.allclose(Ws, frames_seen, rtol=1e-12)


def test_image_weighting_known_two_frame_case():
    """Frame 0 sees texel 0 with 9 pixels of q0, frame 1 with 1 pixel of q1:
    w^(P) gives (9 q0 + q1)/10, w^(I) gives (q0 + q1)/2."""
    q0 = np.array([0.75, 0.125, 0.125])     # dyadic: sums are exact
    q1 = np.array([0.125, 0.0, 0.875])
    l = np.full((2, 3, 3), -1, np.int32)
    l[0] = 0
    l[1, 1, 1] = 0
    p = np.zeros((2, 3, 3, 3), np.float32)
    p[0] = q0
    p[1] = q1
    pn = np.ascontiguousarray(p.transpose(0, 3, 1, 2))
    A, Ws = oracle.fuse(1, 3, l, pn, weighting=oracle.W_PIXEL)
    P, lab = oracle.finalize(A, Ws)
    assert np.allclose(P[0], (9 * q0 + q1) / 10, rtol=1e-12)
    assert lab[0] == 0
    A, Ws = oracle.fuse(1, 3, l, pn, weighting=oracle.W_IMAGE)
    P, lab = oracle.finalize(A, Ws)
    assert np.allclose(P[0], (q0 + q1) / 2, rtol=1e-12)
    assert lab[0] == 2


def test_permutation_invariance_and_incremental():
    """Section 3.3.2: the aggregator is permutation invariant (up to rounding);
    fusing A then B equals fusing A and B together (checkpoint / resume)."""
    c, n, F = 6, 40, 8
    l, valid = _frames(F, 12, 12, n, invalid=0.1)
    p = np.ascontiguousarray(RNG.dirichlet(np.ones(c), size=(F, 12, 12)).astype(np.float32).transpose(0, 3, 1, 2))
    for agg in (oracle.AGG_SUM, oracle.AGG_MUL, oracle.AGG_MAXSUM):
        for wt in (oracle.W_PIXEL, oracle.W_IMAGE):
            A, Ws = oracle.fuse(n, c, l, p, valid, weighting=wt, aggregator=agg)
            perm = RNG.permutation(F)
            A2, W2 = oracle.fuse(n, c, l[perm], p[perm], valid[perm], weighting=wt, aggregator=agg)
            assert np.allclose(A, A2, rtol=1e-12, atol=1e-12)
            A3, W3 = oracle.fuse(n, c, l[:3], p[:3], valid[:3], weighting=wt, aggregator=agg)
            A3, W3 = oracle.fuse(n, c, l[3:], p[3:], valid[3:], weighting=wt, aggregator=agg, A=A3, W_sum=W3)
            assert np.allclose(A, A3, rtol=1e-12, atol=1e-12) and np.allclose(Ws, W3)


def test_mul_and_maxsum_closed_forms():
    """eq. mul: norm of the elementwise product; eq. maxsum: only each
    observation's maximum entry is summed (ties keep every maximal entry)."""
    a = np.array([0.5, 0.3, 0.2], np.float32)
    b = np.array([0.2, 0.2, 0.6], np.float32)
    l = np.zeros((1, 1, 2), np.int32)
    p = np.zeros((1, 3, 1, 2), np.float32)
    p[0, :, 0, 0] = a
    p[0, :, 0, 1] = b
    A, Ws = oracle.fuse(1, 3, l, p, aggregator=oracle.AGG_MUL)
    P, lab = oracle.finalize(A, Ws, aggregator=oracle.AGG_MUL)
    prod = a.astype(np.float64) * b.astype(np.float64)
    assert np.allclose(P[0], prod / prod.sum(), rtol=1e-12)
    assert lab[0] == 2
    # weighted mul: p^w with w^(I) = 1/2 each -> sqrt of the product
    A, Ws = oracle.fuse(1, 3, l, p, aggregator=oracle.AGG_MUL, weighting=oracle.W_IMAGE)
    P, _ = oracle.finalize(A, Ws, aggregator=oracle.AGG_MUL)
    sq = np.sqrt(prod)
    assert np.allclose(P[0], sq / sq.sum(), rtol=1e-12)
    c2 = np.array([0.4, 0.4, 0.2], np.float32)
    p[0, :, 0, 1] = c2
    A, Ws = oracle.fuse(1, 3, l, p, aggregator=oracle.AGG_MAXSUM)
    P, lab = oracle.finalize(A, Ws, aggregator=oracle.AGG_MAXSUM)
    g = np.array([float(np.float32(0.5)) + float(np.float32(0.4)), float(np.float32(0.4)), 0.0])
    assert np.allclose(P[0], g / g.sum(), rtol=1e-12)
    assert lab[0] == 0


def test_strides_nhwc_equal_nchw():
    c, n, F = 5, 20, 3
    l, valid = _frames(F, 6, 7, n)
    p = RNG.dirichlet(np.ones(c), size=(F, 6, 7)).astype(np.float32)   # NHWC memory
    nchw = np.ascontiguousarray(p.transpose(0, 3, 1, 2))
    view = p.transpose(0, 3, 1, 2)                                      # NHWC strides, NCHW indexing
    A1, _ = oracle.fuse(n, c, l, nchw, valid)
    A2, _ = oracle.fuse(n, c, l, view, valid)
    assert np.array_equal(A1, A2)


def test_e4m3_decode_matches_ocp_definition():
    import torch
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([oracle.e4m3_decode(i) for i in range(256)])
    nan = np.isnan(ref)
    assert nan.sum() == 2 and np.array_equal(np.isnan(mine), nan)
    assert np.array_equal(mine[~nan], ref[~nan])
    assert oracle.e4m3_decode(0x7E) == 448.0
    assert oracle.e4m3_decode(0x08) == 2.0 ** -6
    assert oracle.e4m3_decode(0x01) == 2.0 ** -9
    assert oracle.e4m3_decode(0x38) == 1.0


def test_fp8_inputs_dequantise_exactly():
    from paper_2111_11103_amd.scenes import quantize_fp8
    import torch
    c, n, F = 6, 15, 2
    l, valid = _frames(F, 5, 5, n)
    p = torch.from_numpy(RNG.dirichlet(np.ones(c), size=(F, 5, 5)).astype(np.float32)).permute(0, 3, 1, 2).contiguous()
    q, sc = quantize_fp8(p)
    A, _ = oracle.fuse(n, c, l, q.numpy(), valid, scale=sc.numpy())
    deq = (q.view(torch.float8_e4m3fn).to(torch.float64) * sc[:, None].to(torch.float64)).numpy()
    A2, _ = oracle.fuse(n, c, l, deq.astype(np.float32), valid)
    # decode(q) * scale is exact in binary64; compare with binary64 sums of it
    ref = np.zeros((n, c))
    m = (l >= 0) & (valid > 0)
    np.add.at(ref, l[m], deq.transpose(0, 2, 3, 1)[m])
    assert np.allclose(A, ref, rtol=1e-13, atol=0)
    assert np.allclose(A2, ref, rtol=1e-6)


def test_invalid_pixels_and_rows_out_of_range():
    c, n = 3, 4
    l = np.array([[[0, 1], [2, 9]]], np.int32)
    p = np.ones((1, c, 2, 2), np.float32) / 3
    with pytest.raises(ValueError):
        oracle.fuse(n, c, l, p)
    l[0, 1, 1] = 3
    valid = np.array([[[1, 0], [1, 0]]], np.uint8)
    A, Ws = oracle.fuse(n, c, l, p, valid)
    assert list(Ws) == [1.0, 0.0, 1.0, 0.0]
