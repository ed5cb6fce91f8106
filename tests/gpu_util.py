"""Shared helpers for the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from oracle import RenderOpts
from tests import binning_check as BC

IMG_TOL = 1e-4     # images: max |x - ref| / max |ref| per channel group
GRAD_TOL = 1e-3    # gradients: per parameter tensor
EPS_ALPHA = 2e-4   # guard band: relative distance of alpha to alpha_min (FP32 alpha error reaches ~5e-5)
EPS_CLAMP = 2e-4   # ... of o exp(power) to alpha_max (gradient-only decision)
EPS_TERM = 2e-4    # ... of T to T_min
TIE_ULPS = 4       # ... depth gap of two composited neighbours, in float32 ulps


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


def guard_mask(margins, tie_ulps=TIE_ULPS):
    """Pixels whose every compositing decision is clear of its threshold.
    tie_ulps: depth gap (float32 ulps) below which two composited neighbours
    may be ordered either way; 0 where both sides round the same exact depth
    (plain Gaussians: the kernels' depth is the correctly rounded float32 of
    the depth the oracle computes in float64), so that only exact ties
    remain, which both order by index."""
    return ((margins["alpha"] > EPS_ALPHA) & (margins["clamp"] > EPS_CLAMP) & (margins["term"] > EPS_TERM)
            & (margins["tie"] > tie_ulps))


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


def guard_report(margins, tie_ulps=TIE_ULPS):
    """Pixels excluded by the guard band, in total and per threshold."""
    keep = guard_mask(margins, tie_ulps)
    rep = dict(total=int((~keep).sum()), pixels=int(keep.size),
               alpha=int((margins["alpha"] <= EPS_ALPHA).sum()), clamp=int((margins["clamp"] <= EPS_CLAMP).sum()),
               term=int((margins["term"] <= EPS_TERM).sum()), tie=int((margins["tie"] <= tie_ulps).sum()))
    rep["frac"] = rep["total"] / max(1, rep["pixels"])
    return keep, rep


def ctx_binning_state(rc):
    """The context arrays the binning follows from and produces (numpy)."""
    from paper_2505_22335_amd import _lib as L
    ni, nvis, ov = rc.status()
    assert ov == 0, "capacity overflow"
    u32 = lambda a: a.cpu().numpy().view(np.uint32)
    st = dict(n_isect=ni, n_visible=nvis)
    st["geom"] = rc.array(L.CTX_GEOM, torch.float32, width=8).cpu().numpy()
    st["radius"] = rc.array(L.CTX_RADIUS, torch.float32, width=2).cpu().numpy()
    st["dkey"] = u32(rc.array(L.CTX_DEPTH_KEY, torch.int32))
    st["ntiles"] = u32(rc.array(L.CTX_NTILES, torch.int32))
    st["rect"] = rc.array(L.CTX_RECT, torch.int16, width=4).cpu().numpy()
    st["pair_tile"] = u32(rc.array(L.CTX_PAIR_TILE, torch.int32, count=ni)) if ni else np.zeros(0, np.uint32)
    st["pair_gauss"] = u32(rc.array(L.CTX_PAIR_GAUSS, torch.int32, count=ni)) if ni else np.zeros(0, np.uint32)
    st["ranges"] = rc.array(L.CTX_TILE_RANGE, torch.int32, width=2).cpu().numpy()
    return st


def check_binning_self_consistent(rc, label=""):
    """Tile rectangles, sorted pairs and ranges of a context equal their
    integer re-derivation from the kernels' own float32 footprint values, bit
    for bit, with no exclusion."""
    st = ctx_binning_state(rc)
    res = BC.self_consistency(st, [(int(c.width), int(c.height)) for c in rc.cams], rc.n)
    log("binning self-consistency", label, res)
    bad = {k: v for k, v in res.items() if k.endswith("mismatch") or k == "key_invalid"}
    assert all(v == 0 for v in bad.values()), (label, bad)
    return st, res


def check_lists_vs_oracle(rc, ref, st=None, tie_ulps=TIE_ULPS, max_rect_frac=2e-3, max_tie_frac=3e-3, label=""):
    """Cross-precision list check (one view): the kernels' tile lists equal the
    FP64 oracle's once the Gaussians inside the band of an integer decision
    (rectangle edge) or of a depth tie (tie_ulps float32 ulps; 0 for plain
    Gaussians, whose float32 depth both sides round from the same exact value)
    are removed; the number of such Gaussians is reported and bounded."""
    if st is None:
        st = ctx_binning_state(rc)
    p = ref["proj"]
    TX, TY = p["tiles_xy"]
    u = p["u"].detach().numpy()
    v = p["v"].detach().numpy()
    ext = p["extent"]
    rband = BC.rect_band(u, v, ext[:, 0], ext[:, 1], TX, TY) & np.isfinite(ext).all(1)
    # other visibility decisions near their thresholds (depth at znear, opacity at alpha_min)
    z = p["z"].detach().numpy()
    rband |= np.abs(z - 0.2) <= 1e-6 * np.maximum(1.0, np.abs(z))
    tband = BC.tie_band(ref["gids"], ref["ranges"], p["z32"], tie_ulps) if tie_ulps > 0 else set()
    flagged = set(np.flatnonzero(rband).tolist()) | tband
    n_vis = int(p["visible"].sum())
    I = len(ref["gids"])
    gg = st["pair_gauss"].astype(np.int64)
    bad = BC.compare_lists(ref["gids"].astype(np.int64), ref["ranges"].astype(np.int64), gg,
                           st["ranges"].astype(np.int64), np.array(sorted(flagged), np.int64))
    rep = dict(rect_band=int(rband.sum()), tie_band=len(tband), tie_ulps=tie_ulps, visible=n_vis, isect=I,
               gpu_isect=int(st["n_isect"]), tiles_differing=bad)
    log("lists vs oracle", label, rep)
    assert bad == 0, rep
    assert rep["rect_band"] <= max_rect_frac * max(n_vis, 1) + 3, rep
    assert rep["tie_band"] <= max_tie_frac * max(I, 1) + 4, rep
    # the intersection counts differ only by the rectangles inside the band
    return rep
