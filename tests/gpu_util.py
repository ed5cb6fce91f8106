"""Shared helpers for the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from oracle import RenderOpts

IMG_TOL = 1e-4     # images: max |x - ref| / max |ref| per channel group
GRAD_TOL = 1e-3    # gradients: per parameter tensor
EPS_ALPHA = 2e-4   # guard band: relative distance of alpha to alpha_min (FP32 alpha error reaches ~5e-5)
EPS_CLAMP = 2e-4   # ... of o exp(power) to alpha_max (gradient-only decision)
EPS_TERM = 2e-4    # ... of T to T_min
TIE_ULPS = 16      # ... depth gap of two composited neighbours, in float32 ulps


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(x, ref, mask=None):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is not None:
        x = x[..., mask]
        ref = ref[..., mask]
    den = max(np.abs(ref).max() if ref.size else 0.0, 1e-12)
    return float(np.abs(x - ref).max() / den) if ref.size else 0.0


def guard_mask(margins):
    """Pixels whose every compositing decision is clear of its threshold."""
    return ((margins["alpha"] > EPS_ALPHA) & (margins["clamp"] > EPS_CLAMP) & (margins["term"] > EPS_TERM)
            & (margins["tie"] > TIE_ULPS))


def tie_flagged(ref):
    """Gaussians with a tile-list neighbour within TIE_ULPS float32 ulps of depth."""
    z32 = ref["proj"]["z32"]
    gids, rng = ref["gids"], ref["ranges"]
    out = set()
    for s, e in rng:
        if e - s < 2:
            continue
        z = z32[gids[s:e]]
        gap = (z[1:].astype(np.float64) - z[:-1]) / np.spacing(z[:-1]).astype(np.float64)
        for j in np.flatnonzero(gap <= TIE_ULPS):
            out.add(int(gids[s + j]))
            out.add(int(gids[s + j + 1]))
    return out


def upstream(seed, H, W, nf):
    rng = np.random.default_rng(seed)
    G = dict(rgb=rng.normal(size=(3, H, W)), depth=rng.normal(size=(H, W)),
             alpha=rng.normal(size=(H, W)))
    if nf:
        G["feat"] = rng.normal(size=(nf, H, W))
    return {k: v.astype(np.float32) for k, v in G.items()}


def oracle_opts(nf, **kw):
    return RenderOpts(n_feat=nf, **kw)


def to_np(t):
    return t.detach().float().cpu().numpy()
