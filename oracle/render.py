"""The whole hot path in float64: decode -> project -> bin -> composite, and its
backward as the vector-Jacobian product of that forward definition.

Test infrastructure (see the package docstring).

The backward is torch autograd over the float64 forward, run in two stages so
memory stays bounded: per tile, the VJP w.r.t. the 2D records (u, v, conic,
opacity, colour, depth, feature) of the Gaussians in that tile; then one VJP
from the 2D records back through the projection (Eq. 2), the decoder (Eq. 8,
Eq. 9) and the pose twist xi (left perturbation T_cw <- Exp(xi) T_cw).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np
import torch

from .binning import bin_and_sort
from .composite import composite_tile
from .decode import decode
from .geometry import camera_center, pose_cw
from .project import project
from .readings import RenderOpts

F64 = torch.float64


def _t(a, grad=False):
    t = torch.as_tensor(np.asarray(a, dtype=np.float64)).clone()
    if grad:
        t.requires_grad_(True)
    return t


def gaussians_from_plain(scene, grad=False) -> Dict[str, torch.Tensor]:
    """(N, c) float64 leaf tensors from a plain scene's [c][n] float32 planes."""
    g = dict(mean=_t(scene.mean.T, grad), scale=_t(scene.scale.T, grad),
             rot=_t(scene.rot.T, grad), opacity=_t(scene.opacity, grad),
             rgb=_t(scene.rgb.T, grad))
    if scene.feat is not None:
        g["feat"] = _t(scene.feat.T, grad)
    return g


@dataclass
class Leaves:
    """Leaf tensors of one oracle evaluation (whatever required grad)."""
    xi: Optional[torch.Tensor] = None
    gauss: Dict[str, torch.Tensor] = field(default_factory=dict)     # decoded or plain (N,c)
    anchor: Dict[str, torch.Tensor] = field(default_factory=dict)    # xyz, feat, off
    weights: Dict[str, Dict[str, torch.Tensor]] = field(default_factory=dict)


def render(g: Dict[str, torch.Tensor], R_cw, t_cw, cam, opts: RenderOpts, grad_out=None,
           with_margins=False, impact_T=1e-3, keep_lists=False, structure=None, keep_structure=False):
    """Render one view of Gaussians g ((N,c) float64 tensors).

    cam: object with width, height, fx, fy, cx, cy. grad_out: optional dict of
    upstream gradients (numpy) 'rgb' (3,H,W), 'depth' (H,W), 'feat'
    (F,H,W), 'alpha' (H,W); when given, gradients are accumulated into the
    .grad of whatever leaves g was built from.

    Returns a dict of numpy images (rgb, depth, feat, alpha, T_final,
    n_contrib) plus the projection and tile lists.

    keep_structure returns, under 'structure', the tile lists and every
    compositing decision of this evaluation; passing that back as structure
    evaluates the same lists with the same decisions at other inputs
    (frozen-structure finite differences).
    """
    W, H = cam.width, cam.height
    p = project(g["mean"], g["scale"], g["rot"], g["opacity"], R_cw, t_cw, W, H,
                cam.fx, cam.fy, cam.cx, cam.cy, opts)
    nf = g["feat"].shape[1] if ("feat" in g and opts.n_feat > 0) else 0
    parts = [g["rgb"], p["z"][:, None]]
    if nf:
        parts.append(g["feat"])
    chans = torch.cat(parts, 1)
    Cc = chans.shape[1]
    names2d = ["u", "v", "A", "B", "C"]
    src2d = [p[k] for k in names2d] + [g["opacity"], chans]
    lv = [s.detach().clone().requires_grad_(grad_out is not None) for s in src2d]
    TX, TY = p["tiles_xy"]
    if structure is not None:
        tiles, gids, ranges = structure["tiles"], structure["gids"], structure["ranges"]
    else:
        tiles, gids, ranges = bin_and_sort(p["rect"], p["z32"], p["visible"], TX, TY)
    decisions = {}

    acc = np.zeros((H * W, Cc))
    asum = np.zeros(H * W)
    Tfin = np.ones(H * W)
    ncon = np.zeros(H * W, np.int64)
    marg = {k: np.full(H * W, np.inf) for k in ("alpha", "clamp", "term", "tie")}
    if grad_out is not None:
        Gimg = [np.asarray(grad_out["rgb"], np.float64).reshape(3, -1),
                np.asarray(grad_out["depth"], np.float64).reshape(1, -1)]
        if nf:
            Gimg.append(np.asarray(grad_out["feat"], np.float64).reshape(nf, -1))
        Gacc = torch.as_tensor(np.concatenate(Gimg, 0).T.copy())          # (HW, Cc)
        Ga = torch.as_tensor(np.asarray(grad_out.get("alpha", np.zeros((H, W))),
                                        np.float64).reshape(-1).copy())
        bg = torch.as_tensor(np.asarray(opts.bg, np.float64))
        GT = Gacc[:, :3] @ bg                                               # d/dT_final via bg

    T = opts.tile
    ly, lx = np.meshgrid(np.arange(T), np.arange(T), indexing="ij")
    ly, lx = ly.ravel(), lx.ravel()
    for t in range(TX * TY):
        s, e = ranges[t]
        ty, tx = divmod(t, TX)
        pxs = tx * T + lx
        pys = ty * T + ly
        inside = (pxs < W) & (pys < H)
        pxs, pys = pxs[inside], pys[inside]
        pix = pys * W + pxs
        if e == s:
            continue
        ids = torch.as_tensor(gids[s:e])
        args = [x[ids] for x in lv]
        sink = [] if keep_structure else None
        res = composite_tile(*args, torch.as_tensor(pxs, dtype=F64), torch.as_tensor(pys, dtype=F64),
                             opts, with_margins=with_margins and structure is None, impact_T=impact_T,
                             z32=p["z32"][gids[s:e]],
                             frozen=None if structure is None else structure["decisions"][t],
                             structure_out=sink)
        if keep_structure:
            decisions[t] = sink[0]
        a_, s_, T_, n_ = res[:4]
        acc[pix] = a_.detach().numpy()
        asum[pix] = s_.detach().numpy()
        Tfin[pix] = T_.detach().numpy()
        ncon[pix] = n_
        if with_margins and structure is None:
            for k in marg:
                marg[k][pix] = res[4][k]
        if grad_out is not None:
            pt = torch.as_tensor(pix)
            loss = (a_ * Gacc[pt]).sum() + (s_ * Ga[pt]).sum() + (T_ * GT[pt]).sum()
            if loss.requires_grad:
                loss.backward()
    if grad_out is not None:
        outs, grads = [], []
        for s_, l_ in zip(src2d, lv):
            if s_.requires_grad and l_.grad is not None:
                outs.append(s_)
                grads.append(l_.grad)
        if outs:
            torch.autograd.backward(outs, grads)

    rgb = (acc[:, :3] + Tfin[:, None] * np.asarray(opts.bg)[None, :]).T.reshape(3, H, W)
    out = dict(rgb=rgb, depth=acc[:, 3].reshape(H, W), alpha=asum.reshape(H, W),
               T_final=Tfin.reshape(H, W), n_contrib=ncon.reshape(H, W), proj=p,
               grad2d={n: (l.grad.detach().numpy() if l.grad is not None else None)
                       for n, l in zip(names2d + ["o", "chans"], lv)})
    if nf:
        out["feat"] = acc[:, 4:].T.reshape(nf, H, W)
    if with_margins:
        out["margins"] = {k: v.reshape(H, W) for k, v in marg.items()}
    if keep_lists:
        out["tiles"], out["gids"], out["ranges"] = tiles, gids, ranges
    if keep_structure:
        out["structure"] = dict(tiles=tiles, gids=gids, ranges=ranges, decisions=decisions)
    return out


def render_scene(scene, cam, opts: RenderOpts, grad_out=None, pose_grad=False,
                 precision="fp64", with_margins=False, impact_T=1e-3, keep_lists=False,
                 xi0=None, structure=None, keep_structure=False):
    """Evaluate a plain scene (synth.PlainScene) or an anchor scene
    (synth.AnchorScene) at camera cam (synth.Camera).

    With grad_out, returns (images, grads) where grads holds numpy gradients
    of every input: Gaussian planes ([c][n] like the inputs), anchor inputs,
    head weights, the decoded Gaussians (anchor scenes) and 'pose' (6,) =
    dL/dxi. xi0 optionally evaluates at Exp(xi0) T_cw (finite differences);
    structure / keep_structure as in render.
    """
    need = grad_out is not None
    xi = torch.zeros(6, dtype=F64, requires_grad=need and pose_grad)
    if xi0 is not None:
        xi = (xi + torch.as_tensor(np.asarray(xi0, np.float64))).detach().requires_grad_(need and pose_grad)
    R_cw, t_cw = pose_cw(np.asarray(cam.T_wc, np.float64), xi)
    lv = Leaves(xi=xi)
    if hasattr(scene, "xyz"):
        lv.anchor = dict(xyz=_t(scene.xyz.T, need), feat=_t(scene.feat, need),
                         off=_t(scene.off.T, need))
        lv.weights = {h: {k: _t(v, need) for k, v in w.items()} for h, w in scene.weights.items()}
        c = camera_center(R_cw, t_cw)
        g = decode(lv.anchor["xyz"], lv.anchor["feat"], lv.anchor["off"], lv.weights, c,
                   scene.k, scene.l_o, scene.l_s, precision=precision, t=getattr(cam, "t", 0.0))
        if need:
            for v in g.values():
                v.retain_grad()
        lv.gauss = g
    else:
        g = gaussians_from_plain(scene, need)
        lv.gauss = g
    out = render(g, R_cw, t_cw, cam, opts, grad_out=grad_out, with_margins=with_margins,
                 impact_T=impact_T, keep_lists=keep_lists, structure=structure,
                 keep_structure=keep_structure)
    out["gauss"] = {k: v.detach().numpy().T.copy() for k, v in g.items()}
    if not need:
        return out
    grads = {}

    def gr(t):
        return None if t.grad is None else t.grad.detach().numpy()

    grads["gauss"] = {k: (None if v.grad is None else v.grad.detach().numpy().T.copy())
                      for k, v in g.items()}
    if lv.anchor:
        grads["anchor"] = {k: gr(v) for k, v in lv.anchor.items()}
        grads["anchor"]["xyz"] = grads["anchor"]["xyz"].T.copy()
        grads["anchor"]["off"] = grads["anchor"]["off"].T.copy()
        grads["weights"] = {h: {k: gr(v) for k, v in w.items()} for h, w in lv.weights.items()}
    if pose_grad:
        grads["pose"] = gr(xi)
    return out, grads
