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
