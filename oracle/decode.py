"""Anchor -> neural Gaussian decoding (Sec. 3.3, Eq. 8 and Eq. 9).

Test infrastructure (see the package docstring).

Each anchor v carries a position x_v, a 32-d feature f_v and k offsets O_vi.
Its k Gaussians are decoded by five separate two-layer MLPs (opacity, colour,
scale, rotation, low-dimensional feature), each fed with the anchor feature
and the unit direction from the camera centre to the anchor (Eq. 8); the
scene-variant decoders also take the anchor's distance to the camera centre
and the temporal embedding l_t = (sin pi t, cos pi t) of the frame time t
(Sec. 3.3, Temporal Encoding; inputs of Eq. 8 and Eq. 9). The
feature decoder F_d is Linear -> SoftPlus -> Linear with a 32-wide hidden
layer (appendix, MLP details); the other four use ReLU as in Scaffold-GS.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np
import torch
import torch.nn.functional as F

F64 = torch.float64

# (head name, values per Gaussian, hidden activation)
HEAD_ORDER = (
    ("opacity", 1, "relu"),
    ("rgb", 3, "relu"),
    ("scale", 3, "relu"),
    ("rot", 4, "relu"),
    ("feat", 16, "softplus"),
)


def _bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (nearest-even, via float32) and return as float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(F64)


def decode(xyz: torch.Tensor, feat: torch.Tensor, off: torch.Tensor,
           weights: Dict[str, Dict[str, torch.Tensor]], cam_center: torch.Tensor,
           k: int, l_o: float = 1.0, l_s: float = 0.02, precision: str = "fp64", t: float = 0.0):
    """Decode anchors into Gaussians.

    xyz (A,3), feat (A,32), off (A*k,3) row n = v*k+i; weights[head] =
    {W1 (32,in_dim), b1 (32), W2 (k*m,32), b2 (k*m)}; cam_center (3,).
    The input of every head is X = [f_v (32), delta (3)] for in_dim 35,
    followed by the distance |x_v - c| for in_dim 36, and by sin(pi t),
    cos(pi t) as well for in_dim 38 (t the frame time of the view).
    precision 'bf16' rounds the feature-part operands of layer 1 and both
    operands of layer 2 to bfloat16 (what the matrix-core variant feeds its
    MFMAs); sums, biases, the other input columns and activations stay exact.

    Returns dict of (N, c) float64 tensors: mean, scale, rot, opacity (N,),
    rgb, [feat].
    """
    A = xyz.shape[0]
    D = xyz - cam_center[None, :]
    dist = torch.linalg.norm(D, dim=1, keepdim=True)
    delta = D / dist
    # the input columns after the anchor feature, by their number
    lt = torch.tensor([[math.sin(math.pi * t), math.cos(math.pi * t)]], dtype=F64).expand(A, 2)
    extra = {3: [delta], 4: [delta, dist], 6: [delta, dist, lt]}
    out = {}
    for name, m, act in HEAD_ORDER:
        if name not in weights:
            continue
        w = weights[name]
        W1, b1, W2, b2 = w["W1"], w["b1"], w["W2"], w["b2"]
        nf = feat.shape[1]
        if W1.shape[1] - nf not in extra:
            raise ValueError("decoder input width must be 35, 36 or 38 (got %d)" % W1.shape[1])
        rest = torch.cat(extra[W1.shape[1] - nf], 1)
        if precision == "bf16":
            Z = _bf16(feat) @ _bf16(W1[:, :nf]).T + rest @ W1[:, nf:].T + b1
        else:
            Z = torch.cat([feat, rest], 1) @ W1.T + b1
        H = torch.relu(Z) if act == "relu" else F.softplus(Z, beta=1.0, threshold=1e9)
        if precision == "bf16":
            Y = _bf16(H) @ _bf16(W2).T + b2
        else:
            Y = H @ W2.T + b2
        mh = W2.shape[0] // k
        out[name] = Y.reshape(A * k, mh)
    g = {}
    g["mean"] = xyz.repeat_interleave(k, dim=0) + l_o * off
    g["opacity"] = torch.sigmoid(out["opacity"][:, 0])
    g["rgb"] = torch.sigmoid(out["rgb"])
    g["scale"] = l_s * torch.sigmoid(out["scale"])
    g["rot"] = out["rot"]
    if "feat" in out:
        g["feat"] = out["feat"]
    return g


def _bf16_hidden(xyz, feat, weights, cam_center, t):
    """Per head: the bf16 variant's single-precision-exact hidden activations
    H (A, 32), the margin of each to the nearest bfloat16 rounding midpoint
    relative to the sum of |terms| of Z (inf where H = 0), and the bfloat16
    spacing around H."""
    A = xyz.shape[0]
    D = xyz - cam_center[None, :]
    dist = torch.linalg.norm(D, dim=1, keepdim=True)
    delta = D / dist
    lt = torch.tensor([[math.sin(math.pi * t), math.cos(math.pi * t)]], dtype=F64).expand(A, 2)
    extra = {3: [delta], 4: [delta, dist], 6: [delta, dist, lt]}
    out = {}
    for name, m, act in HEAD_ORDER:
        if name not in weights:
            continue
        W1, b1 = weights[name]["W1"].detach(), weights[name]["b1"].detach()
        nf = feat.shape[1]
        rest = torch.cat(extra[W1.shape[1] - nf], 1).detach()
        f16, w16 = _bf16(feat.detach()), _bf16(W1[:, :nf])
        Z = f16 @ w16.T + rest @ W1[:, nf:].T + b1
        scale = f16.abs() @ w16.abs().T + rest.abs() @ W1[:, nf:].abs().T + b1.abs()
        H = torch.relu(Z) if act == "relu" else F.softplus(Z, beta=1.0, threshold=1e9)
        Hn = H.numpy()
        with np.errstate(divide="ignore"):
            e = np.floor(np.log2(np.abs(Hn)))
        ulp = np.where(Hn != 0, np.exp2(e - 7), 0.0)  # spacing of bfloat16 values around H (8 significant bits)
        q = np.abs(Hn) / np.where(Hn != 0, ulp, 1.0)
        d = np.abs((q - np.floor(q)) - 0.5) * ulp
        marg = np.where(Hn != 0, d / np.maximum(scale.numpy(), 1e-300), np.inf)
        out[name] = (Hn, marg, ulp)
    return out


def bf16_hidden_margin(xyz: torch.Tensor, feat: torch.Tensor, weights: Dict[str, Dict[str, torch.Tensor]],
                       cam_center: torch.Tensor, t: float = 0.0):
    """Guard band of the bfloat16 variant's one computed operand: the hidden
    activations H are rounded to bfloat16 after a single-precision first
    layer, so an H within that layer's rounding of a bfloat16 rounding
    midpoint may round either way. Per head, per anchor: the minimum over
    the 32 hidden units of |H - nearest midpoint| / (sum of |terms| of Z),
    with H and Z as in the bf16 mode above (inf where H = 0). Returns
    {head: (A,) float64 numpy array}."""
    return {name: marg.min(axis=1) for name, (_, marg, _) in _bf16_hidden(xyz, feat, weights, cam_center, t).items()}


def bf16_flip_bound(xyz: torch.Tensor, feat: torch.Tensor, weights: Dict[str, Dict[str, torch.Tensor]],
                    cam_center: torch.Tensor, k: int, l_s: float = 0.02, t: float = 0.0, band: float = 2.0 ** -20):
    """Largest change of each decoded value of the bf16 variant that hidden
    units within the guard band (margin < band, see bf16_hidden_margin) can
    cause by rounding the other way: such a unit's bfloat16 operand moves by
    one bfloat16 spacing, which moves the row's pre-activation by that spacing
    times |bf16(W2)| (the products are exact), summed over the unit's
    in-band neighbours of the anchor; the output activations scale it by at
    most their largest slope (1/4 for sigmoid, l_s/4 for the scale head, 1 for
    the raw heads). Returns {head: (A * k, m) float64 numpy array}."""
    slope = dict(opacity=0.25, rgb=0.25, scale=0.25 * l_s, rot=1.0, feat=1.0)
    out = {}
    for name, (_, marg, ulp) in _bf16_hidden(xyz, feat, weights, cam_center, t).items():
        dH = np.where(marg < band, ulp, 0.0)
        W2 = _bf16(weights[name]["W2"].detach()).numpy()
        by = dH @ np.abs(W2).T  # (A, k m)
        m = W2.shape[0] // k
        out[name] = slope[name] * by.reshape(-1, m)
    return out
