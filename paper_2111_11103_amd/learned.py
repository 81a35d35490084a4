"""Training and evaluation driver of the learned per-observation weight.

The weight generalises the fixed w^(P) = 1 and w^(I) = 1/|K_i ∩ K_x| of
Section 3.2.2: w_k = MLP(phi_k).  Training data are the observations of
seeded room scenes (the 2,100-triangle, 13-class, 20-frame 160x120 recipe)
fused plainly (SUM, w^(P)); an observation's target is 1 when its own argmax
equals its texel's plainly fused label.  Every numeric step -- rendering,
features, forward, gradients, Adam -- runs in the library's kernels; this
module only sequences the calls and draws minibatch indices.
"""
from __future__ import annotations

import time

import torch

from . import scenes as S
from . import semfuse as sf


def scene_mesh(w, device):
    sc = w.scene
    return sf.Mesh(torch.as_tensor(sc.vertices, dtype=torch.float32, device=device),
                   torch.as_tensor(sc.faces, dtype=torch.int32, device=device), n_classes=sc.n_classes, s=w.s,
                   scheme=w.scheme)


def scene_observations(w, device="cuda"):
    """(phi [n, 8], target [n]) of one scene against its plain fusion."""
    mesh = scene_mesh(w, device)
    cams = torch.as_tensor(w.cams, dtype=torch.float32, device=device)
    probs = w.probs.to(device)
    valid = w.valid.to(device)
    mesh.fuse_frames(cams, probs, valid=valid, weighting=sf.W_PIXEL)
    _, lab = mesh.finalize(want_tex=False)
    phi, tgt, _ = mesh.extract_features(cams, probs, valid=valid, labels=lab, want_pix=False)
    return phi.clone(), tgt.clone()


def training_set(seeds, device="cuda", structured=True, log=None):
    phis, tgts = [], []
    for sd in seeds:
        w = S.config1(device=device, seed=int(sd), structured=structured)
        phi, tgt = scene_observations(w, device)
        phis.append(phi)
        tgts.append(tgt)
    phi = torch.cat(phis)
    tgt = torch.cat(tgts)
    if log:
        log(f"training set: {len(seeds)} scenes, {phi.shape[0]} observations, "
            f"positive fraction {float(tgt.mean()):.3f}")
    return phi, tgt


def train(mlp: sf.WeightMLP, phi, tgt, steps=400, batch=32768, lr=3e-3, seed=0, log=None, log_every=100):
    """Minibatch Adam on mean binary cross-entropy; returns the loss history
    (one value per logged step)."""
    g = torch.Generator(device=phi.device).manual_seed(int(seed))
    n = phi.shape[0]
    hist = []
    t0 = time.time()
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g, device=phi.device)
        loss, grad = mlp.loss_grad(phi[idx], tgt[idx])
        if it % log_every == 0 or it == steps - 1:
            hist.append(float(loss.item()))
            if log:
                log(f"  step {it:4d}  loss {hist[-1]:.4f}  ({time.time() - t0:.1f} s)")
        mlp.adam(grad, lr=lr)
    return hist


def full_loss(mlp: sf.WeightMLP, phi, tgt):
    loss, _ = mlp.loss_grad(phi, tgt)
    return float(loss.item())


def subsample(w, step: int):
    """The same scene with every ``step``-th frame only."""
    return S.FrameInputs(w.scene, w.cams[::step], w.H, w.W, w.probs[::step], w.valid[::step], w.gt[::step],
                         s=w.s, scheme=w.scheme)


@torch.no_grad()
def evaluate(w, mlp: sf.WeightMLP | None, device="cuda"):
    """Pixel accuracy (rendered fused label == ground truth over valid
    covered pixels) of the input argmax, w^(P), w^(I) and, given ``mlp``,
    the learned weight."""
    cams = torch.as_tensor(w.cams, dtype=torch.float32, device=device)
    probs = w.probs.to(device)
    valid = w.valid.to(device)
    gt = w.gt.to(device)
    res = {}
    l_rows = torch.empty((cams.shape[0], w.H, w.W), dtype=torch.int32, device=device)
    forms = [("pixel", sf.W_PIXEL), ("image", sf.W_IMAGE)]
    if mlp is not None:
        forms.append(("learned", sf.W_LEARNED))
    for name, wt in forms:
        mesh = scene_mesh(w, device)
        if wt == sf.W_LEARNED:
            mesh.bind_mlp(mlp)
        mesh.fuse_frames(cams, probs, valid=valid, weighting=wt, l_out=l_rows)
        _, lab = mesh.finalize(want_tex=False)
        out = mesh.render_labels(lab, l=l_rows, valid=valid)
        seen = (l_rows >= 0) & (valid != 0)
        res[name] = float((out[seen].long() == gt[seen]).float().mean())
        if "input" not in res:
            res["input"] = float((probs.argmax(1)[seen] == gt[seen]).float().mean())
    return res


@torch.no_grad()
def judge(mesh, cams, probs, mlp, *, valid=None, scale=None, holdout_every=5, batch=16,
          scatter_mode=sf.SCATTER_AUTO, margin=0.0):
    """Plain uniform fusion as judge and fallback of the learned weight.

    Every ``holdout_every``-th frame is held out.  The other frames are fused
    twice -- with w^(P) = 1 and with the learned weight -- and each fused
    texture's labels are rendered into the held-out frames and compared with
    those frames' own argmax labels (lf_label_agreement): the label error the
    learned weight is trained to reduce, measured on frames neither fusion
    saw.  The learned weight is kept only when its agreement beats plain
    fusion's by more than ``margin``; otherwise the fallback is w = 1.  The
    mesh's accumulator is left clear.  Returns a dict with ``choice``
    (sf.W_LEARNED or sf.W_PIXEL) and both agreements."""
    F = cams.shape[0]
    if F < 2 or holdout_every < 2:
        raise ValueError("the judge needs at least two frames and holdout_every >= 2")
    dev = probs.device
    ho = (torch.arange(F, device=dev) % holdout_every) == holdout_every - 1
    fi, hi = (~ho).nonzero().squeeze(1), ho.nonzero().squeeze(1)
    cams_f, cams_h = cams[fi].contiguous(), cams[hi].contiguous()
    probs_f, probs_h = probs[fi], probs[hi]
    valid_f = valid_h = scale_f = scale_h = None
    if valid is not None:
        valid_f, valid_h = valid[fi].contiguous(), valid[hi].contiguous()
    if scale is not None:
        scale_f, scale_h = scale[fi].contiguous(), scale[hi].contiguous()
    H, W = probs.shape[2], probs.shape[3]
    l_h = mesh.rasterize(cams_h, H, W, want=("l",))["l"]
    agree = {}
    for name, wt in (("plain", sf.W_PIXEL), ("learned", sf.W_LEARNED)):
        if wt == sf.W_LEARNED:
            mesh.bind_mlp(mlp)
        mesh.reset()
        mesh.fuse_frames(cams_f, probs_f, scale=scale_f, valid=valid_f, weighting=wt, batch=batch,
                         scatter_mode=scatter_mode)
        _, lab = mesh.finalize(want_tex=False)
        img = mesh.render_labels(lab, l=l_h, valid=valid_h)
        n, a = (int(v) for v in sf.label_agreement(probs_h, img, scale=scale_h, valid=valid_h).cpu())
        agree[name] = a / max(n, 1)
    mesh.reset()
    choice = sf.W_LEARNED if agree["learned"] > agree["plain"] + margin else sf.W_PIXEL
    return {"choice": choice, "agreement_plain": agree["plain"], "agreement_learned": agree["learned"],
            "heldout_frames": int(hi.numel()), "fused_frames": int(fi.numel())}
