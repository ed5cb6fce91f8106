"""Seeded per-pixel maps for the residual, feature-lift and loss kernels
(numpy PCG64, float32 outputs, planes [V][C][H][W]).

Stand-ins for what the paper takes from its RGB-D sequences and from DINOv2:
rendered maps, observed colour and depth, and a patch grid of high-dimensional
features that both sides upsample to the image themselves. Only random draws
and layout live here.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))


def residual_maps(seed: int, V: int, H: int, W: int) -> Dict[str, np.ndarray]:
    """Draw order: rendered rgb ~ U[0,1] (V,3,H,W), depth ~ U[0.5,4] (V,H,W),
    opacity sum ~ U[0.75,1] (V,H,W) (about 40 % of pixels above the 0.9
    visibility level), cosine ~ U[-1,1] (V,H,W), observed rgb ~ U[0,1]
    (V,3,H,W), observed depth ~ U[0.5,4] (V,H,W)."""
    rng = np.random.default_rng(seed)
    out = dict(rgb=rng.uniform(0, 1, (V, 3, H, W)), depth=rng.uniform(0.5, 4.0, (V, H, W)),
               alpha=rng.uniform(0.75, 1.0, (V, H, W)), cosine=rng.uniform(-1.0, 1.0, (V, H, W)),
               obs_rgb=rng.uniform(0, 1, (V, 3, H, W)), obs_depth=rng.uniform(0.5, 4.0, (V, H, W)))
    return {k: _f32(v) for k, v in out.items()}


def feature_inputs(seed: int, V: int, H: int, W: int, grid_h: int, grid_w: int, n_high: int = 384):
    """Draw order: rendered features F~ ~ N(0, 0.5) (V,16,H,W); F_m weights
    with the default bounds of a 1x1 convolution, U(+-1/sqrt(fan_in)): W1
    (128,16), b1 (128), W2 (n_high,128), b2 (n_high); DINO patch features
    ~ N(0, 1) (V, n_high, grid_h, grid_w); upstream gradient of the cosine
    map ~ N(0, 1) (V,H,W)."""
    rng = np.random.default_rng(seed)
    feat = rng.normal(0.0, 0.5, (V, 16, H, W))
    W1 = rng.uniform(-0.25, 0.25, (128, 16))
    b1 = rng.uniform(-0.25, 0.25, 128)
    k = 1.0 / np.sqrt(128.0)
    W2 = rng.uniform(-k, k, (n_high, 128))
    b2 = rng.uniform(-k, k, n_high)
    dino = rng.normal(0.0, 1.0, (V, n_high, grid_h, grid_w))
    d_cos = rng.normal(0.0, 1.0, (V, H, W))
    return {k_: _f32(v) for k_, v in dict(feat=feat, W1=W1, b1=b1, W2=W2, b2=b2, dino=dino, d_cos=d_cos).items()}
