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


def mapping_maps(seed: int, V: int, H: int, W: int) -> Dict[str, np.ndarray]:
    """Maps for the mapping loss. The observed colour is a smooth random field
    (a sum of eight 2D cosines per channel, values in [0, 1]) and the rendered
    colour that field plus N(0, 0.05) noise, clipped to [0, 1], so that the
    SSIM window sees structure and a partial match. Draw order: per view and
    channel 8 x (amplitude U[0,0.5], frequencies U[0,0.3] rad/px in y and x,
    phase U[0,2pi]); rendered noise N(0,0.05) (V,3,H,W); observed depth
    U[0.5,4] (V,H,W); rendered depth = observed + N(0,0.05); cosine U[-1,1]
    (V,H,W); motion mask: U[0,1] < 0.2 (V,H,W)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    obs = np.zeros((V, 3, H, W))
    for v in range(V):
        for c in range(3):
            f = np.zeros((H, W))
            for _ in range(8):
                a, fy, fx, ph = rng.uniform(0, 0.5), rng.uniform(0, 0.3), rng.uniform(0, 0.3), rng.uniform(0, 2 * np.pi)
                f += a * np.cos(fy * yy + fx * xx + ph)
            lo, hi = f.min(), f.max()
            obs[v, c] = (f - lo) / max(hi - lo, 1e-9)
    rgb = np.clip(obs + rng.normal(0.0, 0.05, (V, 3, H, W)), 0.0, 1.0)
    od = rng.uniform(0.5, 4.0, (V, H, W))
    dep = od + rng.normal(0.0, 0.05, (V, H, W))
    cos = rng.uniform(-1.0, 1.0, (V, H, W))
    dyn = (rng.uniform(size=(V, H, W)) < 0.2).astype(np.uint8)
    out = {k: _f32(v) for k, v in dict(rgb=rgb, depth=dep, obs_rgb=obs, obs_depth=od, cosine=cos).items()}
    out["dynamic"] = dyn
    return out


def uncertainty_inputs(seed: int, V: int, H: int, W: int, grid_h: int, grid_w: int, n_high: int = 384):
    """Draw order: F_u weights with the default bounds of 1x1 convolutions,
    U(+-1/sqrt(fan_in)): W1 (128, n_high), b1 (128), w2 (128), b2 (1); DINO
    patch features ~ N(0, 1) (V, n_high, grid_h, grid_w); residual
    R = U[0,1]^2 (V,H,W) with 30 % of the pixels set to 0 (the ones the
    visibility mask of Eq. 6 removes)."""
    rng = np.random.default_rng(seed)
    k1, k2 = 1.0 / np.sqrt(n_high), 1.0 / np.sqrt(128.0)
    W1 = rng.uniform(-k1, k1, (128, n_high))
    b1 = rng.uniform(-k1, k1, 128)
    w2 = rng.uniform(-k2, k2, 128)
    b2 = rng.uniform(-k2, k2, 1)
    dino = rng.normal(0.0, 1.0, (V, n_high, grid_h, grid_w))
    R = rng.uniform(0, 1, (V, H, W)) ** 2
    R[rng.uniform(size=(V, H, W)) < 0.3] = 0.0
    return {k: _f32(v) for k, v in dict(W1=W1, b1=b1, w2=w2, b2=b2, dino=dino, R=R).items()}
