"""EWA projection of 3D Gaussians to 2D conics (Sec. 3.1, Eq. 2).

Test infrastructure (see the package docstring).

Sigma = R S S^T R^T with R from the normalised quaternion and S = diag(s)
(Sec. 3.1). The camera-space mean is t = R_cw mu + t_cw; the 2D covariance is
Sigma' = J R_cw Sigma R_cw^T J^T + dilation I, J the Jacobian of the
perspective map at t (Eq. 2). The conic is Sigma'^-1. The footprint is the
tight axis-aligned box of the ellipse on which o exp(-1/2 d^T Sigma'^-1 d)
equals alpha_min, rounded up to whole pixels, and the tile rectangle is
computed from it with integer arithmetic.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .geometry import quat_to_rotmat
from .readings import RenderOpts

F64 = torch.float64


def project(mean, scale, rot, opacity, R_cw, t_cw, width, height, fx, fy, cx, cy,
            opts: RenderOpts):
    """Project N Gaussians ((N,3) mean/scale, (N,4) rot, (N,) opacity).

    Returns a dict with differentiable (N,) tensors u, v, A, B, C (conic
    entries: power = -1/2 (A dx^2 + C dy^2) - B dx dy), z (camera depth) and
    non-differentiable numpy arrays: visible (bool), rect (N,4) int64
    [tx0, tx1, ty0, ty1] inclusive, ntiles, z32 (float32 depth key), and the
    guard-band margin of the footprint radius (distance of its real value
    to the nearest integer), the whole-pixel radii and their unrounded
    values (extent).
    """
    N = mean.shape[0]
    t = mean @ R_cw.T + t_cw[None, :]
    tz_raw = t[:, 2]
    front = (tz_raw > opts.znear).detach()
    tz = torch.where(front, tz_raw, torch.ones_like(tz_raw))
    tx, ty = t[:, 0], t[:, 1]

    qn = rot / torch.linalg.norm(rot, dim=1, keepdim=True)
    R = quat_to_rotmat(qn)
    M = R * scale[:, None, :]
    Sigma = M @ M.transpose(1, 2)

    xr, yr = tx / tz, ty / tz
    if opts.fov_clamp > 0:
        limx = opts.fov_clamp * width / (2.0 * fx)
        limy = opts.fov_clamp * height / (2.0 * fy)
        xr = torch.clamp(xr, -limx, limx)
        yr = torch.clamp(yr, -limy, limy)
    xc, yc = xr * tz, yr * tz
    zero = torch.zeros_like(tz)
    J = torch.stack([
        torch.stack([fx / tz, zero, -fx * xc / (tz * tz)], -1),
        torch.stack([zero, fy / tz, -fy * yc / (tz * tz)], -1),
    ], -2)  # (N,2,3)
    T = J @ R_cw[None, :, :]
    cov = T @ Sigma @ T.transpose(1, 2)
    a = cov[:, 0, 0] + opts.dilation
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + opts.dilation
    det = a * c - b * b
    okdet = (det > 0).detach()
    det_s = torch.where(okdet, det, torch.ones_like(det))
    A = c / det_s
    B = -b / det_s
    C = a / det_s
    u = fx * tx / tz + cx
    v = fy * ty / tz + cy

    # footprint and tile rectangle (integer decisions, not differentiated)
    o = opacity.detach().numpy()
    an = a.detach().numpy()
    cn = c.detach().numpy()
    un = u.detach().numpy()
    vn = v.detach().numpy()
    with np.errstate(divide="ignore", invalid="ignore"):
        kap2 = 2.0 * np.log(o / opts.alpha_min)
        okop = o > opts.alpha_min
        kap2 = np.where(okop, kap2, 0.0)
        if getattr(opts, "extent_mode", 0) == 0:
            # tight box of the ellipse where alpha = alpha_min
            sx = np.sqrt(kap2 * np.maximum(an, 0.0))
            sy = np.sqrt(kap2 * np.maximum(cn, 0.0))
        else:
            # square of three standard deviations along the major axis
            bn = b.detach().numpy()
            mid = 0.5 * (an + cn)
            lmax = mid + np.sqrt(np.maximum(0.1, mid * mid - (an * cn - bn * bn)))
            sx = sy = 3.0 * np.sqrt(np.maximum(lmax, 0.0))
    rx = np.ceil(sx)
    ry = np.ceil(sy)
    margin_r = np.minimum(np.abs(sx - np.round(sx)), np.abs(sy - np.round(sy)))
    Tn = opts.tile
    TX = -(-width // Tn)
    TY = -(-height // Tn)
    vis = front.numpy() & okdet.numpy() & okop & np.isfinite(un) & np.isfinite(vn)
    iu = np.floor(np.where(vis, un, 0.0))
    iv = np.floor(np.where(vis, vn, 0.0))
    tx0 = np.maximum(0.0, np.floor((iu - rx) / Tn))
    tx1 = np.minimum(TX - 1.0, np.floor((iu + rx) / Tn))
    ty0 = np.maximum(0.0, np.floor((iv - ry) / Tn))
    ty1 = np.minimum(TY - 1.0, np.floor((iv + ry) / Tn))
    vis &= (tx0 <= tx1) & (ty0 <= ty1)
    rect = np.stack([tx0, tx1, ty0, ty1], 1).astype(np.int64)
    rect[~vis] = 0
    ntiles = np.where(vis, (rect[:, 1] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 2] + 1), 0)
    z32 = tz_raw.detach().numpy().astype(np.float32)
    return dict(u=u, v=v, A=A, B=B, C=C, z=tz_raw, visible=vis, rect=rect,
                ntiles=ntiles.astype(np.int64), z32=z32, margin_r=margin_r,
                radius=np.stack([rx, ry], 1), extent=np.stack([sx, sy], 1), tiles_xy=(TX, TY))
