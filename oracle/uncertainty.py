"""Multi-modal tracking residual and per-pixel uncertainty (Sec. 3.2 Eq. 6,
Sec. 3.4 Eq. 15) in float64 (test infrastructure, see the package docstring).

Residual (Eq. 6), per pixel of one view:
  R = vis * (l1 sum_c |C~_c - C_c| + l2 |D~ - (D (x) B)| + l3 min(1, 1 - cos(F, F^)))
with B the 3x3 box filter applied to the observed depth, cos the cosine of
the DINO feature F and the rendered high-dimensional feature F^, and vis the
visibility mask of the rendered opacity sum.

Uncertainty (Eq. 15): sigma minimises (1/HW) sum 1/2 (R / sigma^2 + log sigma)
pixel by pixel; the motion mask marks pixels whose uncertainty exceeds a
threshold. Readings where the paper is silent are listed in
``oracle.readings.RESIDUAL_READINGS``.
"""
from __future__ import annotations

import numpy as np

# Residual weights lambda_1^t, lambda_2^t, lambda_3^t (appendix, implementation details).
RESIDUAL_WEIGHTS = (0.25, 0.7, 0.1)


def box3(D: np.ndarray) -> np.ndarray:
    """3x3 box filter of an (H, W) map: the mean of the pixel and its
    neighbours that lie inside the image."""
    D = np.asarray(D, np.float64)
    H, W = D.shape
    s = np.zeros((H, W))
    n = np.zeros((H, W))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ys0, ys1 = max(0, -dy), min(H, H - dy)
            xs0, xs1 = max(0, -dx), min(W, W - dx)
            s[ys0:ys1, xs0:xs1] += D[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
            n[ys0:ys1, xs0:xs1] += 1.0
    return s / n


def cosine(F: np.ndarray, Fh: np.ndarray, eps: float = 1e-12) -> np.ndarray:
    """Per-pixel cosine of two (C, H, W) feature maps, F . Fh / (|F| |Fh|),
    with the norm product bounded below by eps."""
    F = np.asarray(F, np.float64)
    Fh = np.asarray(Fh, np.float64)
    dot = (F * Fh).sum(0)
    nn = np.sqrt((F * F).sum(0)) * np.sqrt((Fh * Fh).sum(0))
    return dot / np.maximum(nn, eps)


def residual(rgb, depth, alpha, cos, obs_rgb, obs_depth, weights=RESIDUAL_WEIGHTS, vis_T=0.1):
    """Eq. 6 for one view. rgb, obs_rgb (3, H, W); depth, alpha, cos,
    obs_depth (H, W). alpha is the rendered opacity sum (Eq. 3), so the
    remaining transmittance is 1 - alpha and a pixel contributes when it is
    below vis_T. Returns R (H, W)."""
    l1, l2, l3 = weights
    rgb = np.asarray(rgb, np.float64)
    obs_rgb = np.asarray(obs_rgb, np.float64)
    vis = (1.0 - np.asarray(alpha, np.float64)) < vis_T
    r_c = np.abs(rgb - obs_rgb).sum(0)
    r_d = np.abs(np.asarray(depth, np.float64) - box3(obs_depth))
    r_f = np.minimum(1.0, 1.0 - np.asarray(cos, np.float64))
    return np.where(vis, l1 * r_c + l2 * r_d + l3 * r_f, 0.0)


def uncertainty(R, sigma_min=1e-3, dyn_thresh=1.0):
    """Eq. 15 pixel by pixel. The objective 1/2 (R / s^2 + log s) falls for
    s < sqrt(2R) and rises after it, so its minimiser over s >= sigma_min is
    max(sigma_min, sqrt(2R)). Returns (sigma (H, W), xi = the mean of the
    objective at sigma, dynamic (H, W) bool = 2 sigma^2 > dyn_thresh)."""
    R = np.asarray(R, np.float64)
    sigma = np.maximum(sigma_min, np.sqrt(2.0 * R))
    obj = 0.5 * (R / sigma ** 2 + np.log(sigma))
    # 2 sigma^2 = 2 max(sigma_min^2, 2R), compared without the rounding of the square root
    dynamic = 2.0 * np.maximum(sigma_min * sigma_min, 2.0 * R) > dyn_thresh
    return sigma, float(obj.mean()), dynamic
