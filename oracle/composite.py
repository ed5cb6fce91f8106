"""Front-to-back alpha compositing (Sec. 3.1 Eq. 3, Sec. 3.3 Eq. 10).

Test infrastructure (see the package docstring).

For a pixel p and its depth-ordered Gaussians, with d = (u - px, v - py),
  power_i = -1/2 (A dx^2 + C dy^2) - B dx dy,
  alpha_i = min(alpha_max, o_i exp(power_i)),
a Gaussian with power_i > 0 or alpha_i < alpha_min is skipped; otherwise
T' = T (1 - alpha_i); if T' < T_min compositing stops before i; else the
channels (colour, depth z_i, feature) accumulate with weight alpha_i T and
T = T'. Outputs: C = sum w c + T bg, D = sum w z, F = sum w f, and the opacity
sum alpha = sum w (Eq. 3's accumulated term, equal to 1 - T_final).
"""
from __future__ import annotations

import numpy as np
import torch

from .readings import RenderOpts

F64 = torch.float64


def composite_tile(u, v, A, B, C, o, chans, px, py, opts: RenderOpts, with_margins=False,
                   impact_T=1e-3, z32=None, frozen=None, structure_out=None):
    """Composite K depth-ordered Gaussians over P pixels, vectorised.

    u, v, A, B, C, o: (K,) tensors; chans: (K, Cc) tensors (colour, depth,
    feature...); px, py: (P,) float64 pixel coordinates. Returns
    (acc (P,Cc), alpha_sum (P,), T_final (P,), n_contrib (P,) numpy int) and,
    if requested, a dict of per-pixel decision margins for the guard band.

    frozen = (keep, clamped), two (K,P) boolean arrays, replaces the three
    compositing decisions (skip below alpha_min, clamp at alpha_max, stop
    below T_min) by the given ones, so that the outputs are a smooth function
    of the inputs near the point where the decisions were taken
    (frozen-structure finite differences). With structure_out (a list), the
    decisions of this call are appended to it in that form.
    """
    if frozen is not None:
        return _composite_frozen(u, v, A, B, C, o, chans, px, py, opts, frozen)
    K = u.shape[0]
    P = px.shape[0]
    if K == 0:
        z = torch.zeros((P, chans.shape[1]), dtype=F64)
        out = (z, torch.zeros(P, dtype=F64), torch.ones(P, dtype=F64), np.zeros(P, np.int64))
        if with_margins:
            return out + (dict(alpha=np.full(P, np.inf), clamp=np.full(P, np.inf),
                               term=np.full(P, np.inf), tie=np.full(P, np.inf)),)
        return out
    dx = u[:, None] - px[None, :]
    dy = v[:, None] - py[None, :]
    power = -0.5 * (A[:, None] * dx * dx + C[:, None] * dy * dy) - B[:, None] * dx * dy
    raw = o[:, None] * torch.exp(power)
    alpha = torch.clamp(raw, max=opts.alpha_max)
    valid = ((power <= 0) & (alpha >= opts.alpha_min)).detach()
    a = torch.where(valid, alpha, torch.zeros_like(alpha))
    om = 1.0 - a
    T_after = torch.cumprod(om, 0)
    T_before = torch.cat([torch.ones((1, P), dtype=F64), T_after[:-1]], 0)
    term = valid & (T_after < opts.T_min).detach()
    stopped = torch.cumsum(term.to(torch.int64), 0) > 0  # at and after the first stop
    keep = valid & ~stopped
    w = torch.where(keep, a * T_before, torch.zeros_like(a))
    acc = w.T @ chans
    alpha_sum = w.sum(0)
    T_final = torch.where(keep, om, torch.ones_like(om)).prod(0)
    kn = keep.numpy()
    idx = np.arange(1, K + 1)[:, None]
    n_contrib = np.max(np.where(kn, idx, 0), axis=0)
    if structure_out is not None:
        structure_out.append((kn.copy(), (raw >= opts.alpha_max).detach().numpy()))
    if not with_margins:
        return acc, alpha_sum, T_final, n_contrib
    # Guard-band margins: relative distance of each decision to its threshold,
    # over the Gaussians a pixel actually reaches (up to and including the one
    # that stops it). An alpha_min (or alpha_max) decision taken where the
    # transmittance is below impact_T cannot move the outputs by more than
    # ~2 alpha_min impact_T times a channel value and is ignored. A
    # termination decision is never ignored: the Gaussian it admits or stops
    # may have any alpha, so its effect is up to T times a channel value.
    with torch.no_grad():
        first_stop = term & (torch.cumsum(term.to(torch.int64), 0) == 1)
        reached_all = ((~stopped) | first_stop).numpy() & (power.numpy() <= 0)
        reached = reached_all & (T_before.numpy() >= impact_T)
        vn = valid.numpy()
        m_alpha = np.where(reached, np.abs(alpha.numpy() - opts.alpha_min) / opts.alpha_min, np.inf)
        m_clamp = np.where(reached & vn, np.abs(raw.numpy() - opts.alpha_max) / opts.alpha_max, np.inf)
        m_term = np.where(reached_all & vn, np.abs(T_after.numpy() - opts.T_min) / opts.T_min, np.inf)
        margins = dict(alpha=m_alpha.min(0), clamp=m_clamp.min(0), term=m_term.min(0),
                       tie=np.full(P, np.inf))
        if z32 is not None and K > 1:
            # depth order of two neighbours both composited at a pixel, in
            # float32 ulps: a near tie may be ordered either way by a float32
            # depth computed with different rounding
            zf = np.asarray(z32, np.float32)
            gap = (zf[1:].astype(np.float64) - zf[:-1]) / np.spacing(zf[:-1]).astype(np.float64)
            both = (reached & vn)[1:] & (reached & vn)[:-1]
            m_tie = np.where(both, gap[:, None], np.inf)
            margins["tie"] = m_tie.min(0)
    return acc, alpha_sum, T_final, n_contrib, margins


def _composite_frozen(u, v, A, B, C, o, chans, px, py, opts: RenderOpts, frozen):
    """Eq. 3 / Eq. 10 with the per-(Gaussian, pixel) decisions given."""
    keep = torch.as_tensor(np.asarray(frozen[0], bool))
    clamped = torch.as_tensor(np.asarray(frozen[1], bool))
    P = px.shape[0]
    dx = u[:, None] - px[None, :]
    dy = v[:, None] - py[None, :]
    power = -0.5 * (A[:, None] * dx * dx + C[:, None] * dy * dy) - B[:, None] * dx * dy
    raw = o[:, None] * torch.exp(power)
    alpha = torch.where(clamped, torch.full_like(raw, opts.alpha_max), raw)
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    om = 1.0 - a
    T_after = torch.cumprod(om, 0)
    T_before = torch.cat([torch.ones((1, P), dtype=F64), T_after[:-1]], 0)
    w = a * T_before
    acc = w.T @ chans
    idx = np.arange(1, keep.shape[0] + 1)[:, None]
    n_contrib = np.max(np.where(keep.numpy(), idx, 0), axis=0)
    return acc, w.sum(0), om.prod(0), n_contrib


def composite_bruteforce(u, v, A, B, C, o, z, chans, width, height, opts: RenderOpts):
    """Per-pixel reference with no tiles and no keys: for every pixel, every
    Gaussian in (depth, index) order, sequential loop. Pure Python; use on
    images of a few thousand pixels and a few hundred Gaussians.

    All arguments are float64 numpy arrays; returns (acc (H,W,Cc), alpha_sum
    (H,W), T_final (H,W), n_contrib (H,W)) where n_contrib counts positions
    in the global depth order (not comparable to tile positions).
    """
    order = sorted(range(len(u)), key=lambda i: (float(z[i]), i))
    Cc = chans.shape[1]
    acc = np.zeros((height, width, Cc))
    asum = np.zeros((height, width))
    Tf = np.ones((height, width))
    for py in range(height):
        for px in range(width):
            T = 1.0
            s = np.zeros(Cc)
            sa = 0.0
            for i in order:
                dx = u[i] - px
                dy = v[i] - py
                power = -0.5 * (A[i] * dx * dx + C[i] * dy * dy) - B[i] * dx * dy
                if power > 0:
                    continue
                al = min(opts.alpha_max, o[i] * np.exp(power))
                if al < opts.alpha_min:
                    continue
                Tn = T * (1.0 - al)
                if Tn < opts.T_min:
                    break
                s += chans[i] * al * T
                sa += al * T
                T = Tn
            acc[py, px] = s
            asum[py, px] = sa
            Tf[py, px] = T
    return acc, asum, Tf
