"""Feature lift F_m and cosine distillation loss (Sec. 3.3, Eq. 11 and Eq. 12)
in float64 (test infrastructure, see the package docstring).

The rendered low-dimensional feature map F~ (N_l = 16 channels, Eq. 10) is
lifted pixel by pixel by F_m, a 1x1 convolution to 128 hidden channels, ReLU,
and a 1x1 convolution to N_h channels (appendix, MLP details), giving F^. The
DINO features F live on a grid of image patches and are upsampled to the
image bilinearly. The distillation loss is the mean over pixels of
1 - cos(F, F^) (Eq. 12); the per-pixel cosine also enters the tracking
residual (Eq. 6). Readings: ``oracle.readings.FEATURE_READINGS``.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def bilinear_weights(n_out: int, n_in: int):
    """Source cells and weights of bilinear upsampling of n_in samples to
    n_out along one axis, with sample centres at half-integers (output i sits
    at input coordinate (i + 0.5) n_in / n_out - 0.5, clamped at 0) and the
    last sample repeated past the end. Returns (i0, i1, w1) int, int, float
    arrays: value = (1 - w1) v[i0] + w1 v[i1]."""
    src = (np.arange(n_out) + 0.5) * (n_in / n_out) - 0.5
    src = np.maximum(src, 0.0)
    i0 = np.floor(src).astype(np.int64)
    i0 = np.minimum(i0, n_in - 1)
    i1 = np.minimum(i0 + 1, n_in - 1)
    w1 = src - i0
    return i0, i1, w1


def upsample(grid, H: int, W: int):
    """(C, Hp, Wp) patch features -> (C, H, W), bilinear as above, written
    out per axis (float64 tensor in, tensor out; differentiable)."""
    grid = torch.as_tensor(grid, dtype=F64)
    C, Hp, Wp = grid.shape
    y0, y1, wy = bilinear_weights(H, Hp)
    x0, x1, wx = bilinear_weights(W, Wp)
    wy = torch.as_tensor(wy)[None, :, None]
    wx = torch.as_tensor(wx)[None, None, :]
    rows = grid[:, y0, :] * (1 - wy) + grid[:, y1, :] * wy          # (C, H, Wp)
    return rows[:, :, x0] * (1 - wx) + rows[:, :, x1] * wx           # (C, H, W)


def lift(Ft, W1, b1, W2, b2):
    """F^ = W2 relu(W1 F~ + b1) + b2 at every pixel. Ft (16, H, W); W1
    (128, 16), b1 (128), W2 (N_h, 128), b2 (N_h). Returns (N_h, H, W)."""
    Ft = torch.as_tensor(Ft, dtype=F64)
    C, H, W = Ft.shape
    X = Ft.reshape(C, H * W)
    Hd = torch.relu(torch.as_tensor(W1, dtype=F64) @ X + torch.as_tensor(b1, dtype=F64)[:, None])
    Y = torch.as_tensor(W2, dtype=F64) @ Hd + torch.as_tensor(b2, dtype=F64)[:, None]
    return Y.reshape(-1, H, W)


def cosine_map(F, Fh, eps: float = 1e-12):
    """Per-pixel cos(F, F^) of (C, H, W) tensors, the product of the norms
    bounded below by eps (differentiable)."""
    dot = (F * Fh).sum(0)
    nn = torch.sqrt((F * F).sum(0)) * torch.sqrt((Fh * Fh).sum(0))
    return dot / torch.clamp(nn, min=eps)


def distill(Ft, W1, b1, W2, b2, grid, d_cos=None):
    """Cosine map and L_d = mean(1 - cos) for one view; with d_cos ((H, W)
    upstream gradient of a loss w.r.t. the cosine map), also the gradients of
    that loss, sum(d_cos * cos), w.r.t. F~ and the F_m parameters (torch
    autograd of this float64 definition). Returns dict(cos, loss[, grads])."""
    need = d_cos is not None
    leaf = lambda a: torch.as_tensor(np.asarray(a, np.float64)).clone().requires_grad_(need)
    Ft_, W1_, b1_, W2_, b2_ = (leaf(a) for a in (Ft, W1, b1, W2, b2))
    H, W = Ft_.shape[1], Ft_.shape[2]
    F = upsample(np.asarray(grid, np.float64), H, W)
    Fh = lift(Ft_, W1_, b1_, W2_, b2_)
    cos = cosine_map(F, Fh)
    out = dict(cos=cos.detach().numpy(), loss=float((1.0 - cos).mean().detach()))
    if need:
        (cos * torch.as_tensor(np.asarray(d_cos, np.float64))).sum().backward()
        out["grads"] = dict(feat=Ft_.grad.numpy(), W1=W1_.grad.numpy(), b1=b1_.grad.numpy(),
                            W2=W2_.grad.numpy(), b2=b2_.grad.numpy())
    return out


def relu_margin(Ft, W1, b1):
    """Per-pixel guard-band margin of the ReLU decisions of F_m's hidden
    layer: min over units of |z_k| / (sum_c |W1_kc x_c| + |b1_k|), the
    distance of the pre-activation to zero relative to the size of its terms
    (a single-precision evaluation can take the decision differently only
    where this is of the order of its rounding). Returns (H, W)."""
    Ft = np.asarray(Ft, np.float64)
    C, H, W = Ft.shape
    X = Ft.reshape(C, H * W)
    W1 = np.asarray(W1, np.float64)
    b1 = np.asarray(b1, np.float64)
    z = W1 @ X + b1[:, None]
    scale = np.abs(W1) @ np.abs(X) + np.abs(b1)[:, None]
    return (np.abs(z) / np.maximum(scale, 1e-300)).min(0).reshape(H, W)
