"""Mapping-loss assembly in float64 (test infrastructure, see the package
docstring): the geometric loss with SSIM (Sec. 3.1, Eq. 4), the uncertainty
MLP F_u and its negative log-likelihood loss (Sec. 3.2 Eq. 5, Sec. 3.3
Eq. 13), the motion mask, and the total mapping loss with the mean-scale term
(Sec. 3.3, Eq. 14).

Per view of H x W pixels, with rendered colour C~ (3, H, W) and depth D~,
observed C and D, the per-pixel cosine cos(F, F^) of the distillation loss
(Eq. 12) and the motion mask M:

  l_p = (1 - M_p) [ lam1 (lam |C~_p - C_p|^2 + (1 - lam)(1 - SSIM_p))
                    + lam2 (D~_p - D_p)^2 + lam4 (1 - cos_p) ]
  L   = mean_p l_p + lam5 * s_bar,     s_bar = mean of the Gaussians' scales

SSIM_p is the mean over the colour channels of the structural-similarity map
with an 11 x 11 Gaussian window (sigma 1.5), zero padding outside the image,
C1 = 0.01^2 and C2 = 0.03^2.

F_u maps the (bilinearly upsampled) DINO feature of each pixel through
N_h -> 128 (ReLU) -> 1 (SoftPlus); sigma = sigma_min + that output. L_u is
the mean over pixels of R / (2 sigma^2) + lam3 log sigma with R the residual
of Eq. 6 held constant, so L_u trains F_u alone and L the Gaussians alone
(the two gradient flows of the mapping iteration are separate). The motion
mask is M = [2 sigma^2 > 1]. Readings: ``oracle.readings.MAPPING_READINGS``.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as Fnn

from .feature import upsample

F64 = torch.float64

# lam, lam1, lam2, lam3, lam4 (appendix, implementation details); lam5 unstated
MAPPING_WEIGHTS = dict(lam=0.8, lam1=0.6, lam2=1.0, lam3=0.4, lam4=0.01, lam5=0.01)
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
SSIM_WIN = 11
SSIM_SIGMA = 1.5


def gaussian_window(size: int = SSIM_WIN, sigma: float = SSIM_SIGMA) -> np.ndarray:
    """Normalised 1D Gaussian taps g[i] ~ exp(-(i - size//2)^2 / (2 sigma^2))."""
    x = np.arange(size) - size // 2
    g = np.exp(-(x * x) / (2.0 * sigma * sigma))
    return g / g.sum()


def gaussian_filter(img, size: int = SSIM_WIN, sigma: float = SSIM_SIGMA):
    """2D Gaussian filter of a (C, H, W) tensor with zero padding (each output
    pixel is the window-weighted sum of the in-image inputs), as one 2D
    convolution with the outer product of the taps."""
    img = torch.as_tensor(img, dtype=F64)
    g = torch.as_tensor(gaussian_window(size, sigma))
    w2 = torch.outer(g, g)[None, None]
    C = img.shape[0]
    return Fnn.conv2d(img[:, None], w2, padding=size // 2).reshape(C, img.shape[1], img.shape[2])


def ssim_map(x, y):
    """Per-channel SSIM map of two (C, H, W) tensors (differentiable)."""
    mx, my = gaussian_filter(x), gaussian_filter(y)
    sxx = gaussian_filter(x * x) - mx * mx
    syy = gaussian_filter(y * y) - my * my
    sxy = gaussian_filter(x * y) - mx * my
    num = (2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)
    den = (mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)
    return num / den


def pixel_loss(rgb, depth, obs_rgb, obs_depth, cos=None, dynamic=None, weights=None):
    """Per-pixel mapping loss l_p of one view (tensors in, (H, W) tensor out;
    differentiable in rgb, depth and cos)."""
    w = dict(MAPPING_WEIGHTS, **(weights or {}))
    rgb = torch.as_tensor(rgb, dtype=F64)
    obs_rgb = torch.as_tensor(obs_rgb, dtype=F64)
    s = ssim_map(rgb, obs_rgb).mean(0)
    col = ((rgb - obs_rgb) ** 2).sum(0)
    dep = (torch.as_tensor(depth, dtype=F64) - torch.as_tensor(obs_depth, dtype=F64)) ** 2
    lp = w["lam1"] * (w["lam"] * col + (1 - w["lam"]) * (1 - s)) + w["lam2"] * dep
    if cos is not None:
        lp = lp + w["lam4"] * (1 - torch.as_tensor(cos, dtype=F64))
    if dynamic is not None:
        lp = lp * (1.0 - torch.as_tensor(np.asarray(dynamic, np.float64)))
    return lp


def mapping_loss(rgb, depth, obs_rgb, obs_depth, cos=None, dynamic=None, weights=None):
    """mean_p l_p of one view and its gradients w.r.t. the rendered colour,
    the rendered depth and the cosine map (torch autograd of the definition).
    Returns dict(loss, d_rgb, d_depth[, d_cos])."""
    leaf = lambda a: torch.as_tensor(np.asarray(a, np.float64)).clone().requires_grad_(True)
    r, d = leaf(rgb), leaf(depth)
    c = leaf(cos) if cos is not None else None
    L = pixel_loss(r, d, obs_rgb, obs_depth, c, dynamic, weights).mean()
    L.backward()
    out = dict(loss=float(L.detach()), d_rgb=r.grad.numpy(), d_depth=d.grad.numpy())
    if c is not None:
        out["d_cos"] = c.grad.numpy()
    return out


def mean_scale(scale) -> float:
    """s_bar: the mean of the linear scales over all Gaussians and axes."""
    return float(np.asarray(scale, np.float64).mean())


def uncertainty_mlp(grid, W1, b1, w2, b2, H: int, W: int, sigma_min: float = 1e-3):
    """sigma (H, W) = sigma_min + softplus(w2 . relu(W1 F_p + b1) + b2) with F_p
    the DINO feature of pixel p bilinearly upsampled from grid (N_h, Hp, Wp).
    W1 (128, N_h), b1 (128), w2 (128), b2 scalar (differentiable)."""
    F = upsample(grid, H, W)
    Nh = F.shape[0]
    X = F.reshape(Nh, H * W)
    h = torch.relu(torch.as_tensor(W1, dtype=F64) @ X + torch.as_tensor(b1, dtype=F64)[:, None])
    y = torch.as_tensor(w2, dtype=F64) @ h + torch.as_tensor(b2, dtype=F64)
    return (sigma_min + Fnn.softplus(y, beta=1.0, threshold=1e9)).reshape(H, W)


def uncertainty_loss(grid, W1, b1, w2, b2, R, sigma_min: float = 1e-3, lam3: float = MAPPING_WEIGHTS["lam3"],
                     need_grad: bool = True):
    """L_u = mean_p R_p / (2 sigma_p^2) + lam3 log sigma_p of one view (R held
    constant), sigma, the motion mask 2 sigma^2 > 1 and, with need_grad, the
    gradients of L_u w.r.t. F_u's parameters. Returns dict(loss, sigma,
    dynamic[, grads])."""
    leaf = lambda a: torch.as_tensor(np.asarray(a, np.float64)).clone().requires_grad_(need_grad)
    W1_, b1_, w2_, b2_ = leaf(W1), leaf(b1), leaf(w2), leaf(b2)
    H, W = np.shape(R)
    sig = uncertainty_mlp(grid, W1_, b1_, w2_, b2_, H, W, sigma_min)
    Rt = torch.as_tensor(np.asarray(R, np.float64))
    L = (Rt / (2 * sig * sig) + lam3 * torch.log(sig)).mean()
    out = dict(loss=float(L.detach()), sigma=sig.detach().numpy(), dynamic=(2 * sig * sig > 1).detach().numpy())
    if need_grad:
        L.backward()
        out["grads"] = dict(W1=W1_.grad.numpy(), b1=b1_.grad.numpy(), w2=w2_.grad.numpy(),
                            b2=float(b2_.grad.numpy()))
    return out


def softplus_inverse(s: float) -> float:
    """y with softplus(y) = s (s > 0), for building cases with a chosen sigma."""
    return s + math.log(-math.expm1(-s))


def uncertainty_flip_bound(grid, W1, b1, w2, b2, R, sigma_min: float = 1e-3, lam3: float = MAPPING_WEIGHTS["lam3"],
                           band: float = 2e-5):
    """Guard band of the ReLU decisions of F_u's hidden layer for one view:
    a (pixel, unit) pair whose pre-activation z lies within band * (sum of
    |terms| of z) of zero may take the other decision in single precision.
    Returns, per parameter of F_u, the sum over such pairs of the magnitude
    of their contribution to dL_u/dparameter (so that any mix of decisions
    moves the gradient by at most this), and the number of pairs:
    dict(W1 (128, N_h), b1 (128), w2 (128), b2 0.0, pairs)."""
    H, W = np.shape(R)
    F = upsample(grid, H, W).numpy().reshape(-1, H * W)
    W1 = np.asarray(W1, np.float64)
    b1 = np.asarray(b1, np.float64)
    w2 = np.asarray(w2, np.float64)
    Z = W1 @ F + b1[:, None]
    near = np.abs(Z) <= band * (np.abs(W1) @ np.abs(F) + np.abs(b1)[:, None])
    y = w2 @ np.maximum(Z, 0.0) + float(b2)
    sig = sigma_min + np.logaddexp(0.0, y)
    Rf = np.asarray(R, np.float64).reshape(-1)
    dy = (-Rf / sig ** 3 + lam3 / sig) / (H * W) / (1.0 + np.exp(-y))
    A = near * np.abs(dy)[None, :] * np.abs(w2)[:, None]
    return dict(W1=A @ np.abs(F).T, b1=A.sum(1), w2=(near * np.abs(dy)[None, :] * np.abs(Z)).sum(1), b2=0.0,
                pairs=int(near.sum()))
