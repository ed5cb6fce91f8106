"""torch.autograd front end of the decode -> render path, with SE(3) pose
gradients for tracking (UP-SLAM Sec. 3.4: the camera pose is optimised
through the rendering loss; the photometric, depth and feature maps are those
of Eq. 3 and Eq. 10).

Pose parametrisation. Each view v has a base pose T_cw,v (world -> camera)
held on the host and a twist xi_v = (rho, phi) in R^6 (translation part
first); the view is rendered at Exp(xi_v^) T_cw,v. The library returns the
gradient g for a left perturbation at the rendered pose,
Exp(delta^) Exp(xi^) T_cw, and the chain rule through
Exp((xi + d xi)^) = Exp((J_l(xi) d xi)^) Exp(xi^) gives
dL/dxi = J_l(xi)^T g with J_l the left Jacobian of SE(3). J_l is the series
sum_n ad(xi)^n / (n+1)! with ad(xi) = [[phi^, rho^], [0, phi^]], evaluated
exactly as the upper-right block of the exponential of [[ad, I], [0, 0]].

The forward reads xi to the host (one small synchronising copy) to place the
cameras; all other work stays on the device. A renderer keeps one
forward/backward context: the backward must follow its own forward before the
renderer's next forward (checked).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np
import scipy.linalg
import torch

from .core import RenderContext
from .pipeline import AnchorRenderer, DeviceAnchors


@dataclass
class PinholeCamera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    T_wc: np.ndarray  # (3, 4) camera -> world, row-major
    t: float = 0.0    # frame time (temporal decoder input)


def hat(w) -> np.ndarray:
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def twist_matrix(xi) -> np.ndarray:
    """4x4 matrix of xi = (rho, phi)."""
    xi = np.asarray(xi, np.float64)
    M = np.zeros((4, 4))
    M[:3, :3] = hat(xi[3:])
    M[:3, 3] = xi[:3]
    return M


def se3_exp(xi) -> np.ndarray:
    return scipy.linalg.expm(twist_matrix(xi))


def se3_ad(xi) -> np.ndarray:
    xi = np.asarray(xi, np.float64)
    ad = np.zeros((6, 6))
    ad[:3, :3] = hat(xi[3:])
    ad[:3, 3:] = hat(xi[:3])
    ad[3:, 3:] = hat(xi[3:])
    return ad


def se3_left_jacobian(xi) -> np.ndarray:
    """J_l(xi) = sum_n ad(xi)^n / (n+1)!, via the exponential of a 12x12 block matrix."""
    M = np.zeros((12, 12))
    M[:6, :6] = se3_ad(xi)
    M[:6, 6:] = np.eye(6)
    return scipy.linalg.expm(M)[:6, 6:]


def T_cw_of(cam) -> np.ndarray:
    T = np.eye(4)
    T[:3, :] = np.asarray(cam.T_wc, np.float64)
    return np.linalg.inv(T)


def camera_at(cam, T_cw: np.ndarray) -> PinholeCamera:
    T_wc = np.linalg.inv(T_cw)[:3, :]
    return PinholeCamera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                         float(cam.cy), np.ascontiguousarray(T_wc, dtype=np.float32), float(getattr(cam, "t", 0.0)))


class TrackedRenderer:
    """An AnchorRenderer whose view poses are base poses times a twist."""

    def __init__(self, anchors: DeviceAnchors, cams: Sequence, precision: int = 0, **opt_kw):
        self.base = [T_cw_of(c) for c in cams]
        self.intr = list(cams)
        self.r = AnchorRenderer(anchors, cams, precision=precision, **opt_kw)
        self.r.fit()
        self.generation = 0

    @property
    def V(self) -> int:
        return len(self.base)

    def set_base_poses(self, T_cw: Sequence[np.ndarray]):
        if len(T_cw) != self.V:
            raise ValueError("number of views is fixed")
        self.base = [np.asarray(T, np.float64) for T in T_cw]

    def poses(self, xi: np.ndarray):
        return [se3_exp(xi[v]) @ self.base[v] for v in range(self.V)]

    def place(self, xi: np.ndarray):
        cams = [camera_at(c, T) for c, T in zip(self.intr, self.poses(xi))]
        self.r.set_cameras(cams)

    def retract(self, xi: np.ndarray):
        """Fold a twist into the base poses (the tracking update)."""
        self.base = self.poses(np.asarray(xi, np.float64))


class _DecodeRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, xyz, feat, off, params, tr: TrackedRenderer, check: bool):
        xi_h = xi.detach().to("cpu", torch.float64).numpy().reshape(tr.V, 6)
        tr.place(xi_h)
        a = tr.r.a
        tr.r.a = DeviceAnchors(xyz=xyz.detach(), feat=feat.detach(), off=off.detach(), params=params.detach(),
                               k=a.k, n_feat=a.n_feat, l_o=a.l_o, l_s=a.l_s)
        tr.r.decode()
        if check:
            need = tr.r.rc.count(tr.r.g)
            if need > tr.r.rc.capacity:
                tr.r.rc.ensure(int(need * 1.25) + 1024)
        img = tr.r.rc.forward(tr.r.g, out=None)
        tr.generation += 1
        ctx.tr, ctx.gen = tr, tr.generation
        ctx.J = torch.as_tensor(np.stack([se3_left_jacobian(x) for x in xi_h]), dtype=torch.float32,
                                device=xi.device)
        ctx.nf = "feat" in img
        ctx.shapes = {k: v.shape for k, v in img.items()}
        outs = (img["rgb"], img["depth"], img["alpha"], img["feat"] if ctx.nf else img["depth"].new_zeros(0))
        return outs

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_alpha, d_feat):
        tr = ctx.tr
        if tr.generation != ctx.gen:
            raise RuntimeError("TrackedRenderer: backward after a newer forward on the same renderer")
        _raise_on_overflow(tr.r.rc)

        def g(x, key):
            return x.contiguous() if x is not None else torch.zeros(ctx.shapes[key], device=tr.r.a.xyz.device)
        dimg = {"rgb": g(d_rgb, "rgb"), "depth": g(d_depth, "depth"), "alpha": g(d_alpha, "alpha")}
        if ctx.nf:
            dimg["feat"] = g(d_feat, "feat")
        out = tr.r.backward(dimg, pose=True)
        d_xi = torch.bmm(ctx.J.transpose(1, 2).contiguous(), out["d_pose"][:, :, None])[:, :, 0]
        return (d_xi, out["d_xyz"], out["d_feat"], out["d_off"], out["d_params"], None, None)


def decode_render(xi: torch.Tensor, xyz: torch.Tensor, feat: torch.Tensor, off: torch.Tensor,
                  params: torch.Tensor, tr: TrackedRenderer, check: bool = True) -> Dict[str, torch.Tensor]:
    """Differentiable decode + render of tr's views at Exp(xi_v) T_cw,v.

    xi: (V, 6) twists (rho, phi); xyz (3, A), feat (A, 32), off (3, A*k),
    params (packed head parameters): float32 device tensors. Returns rgb
    (V,3,H,W), depth (V,H,W), alpha (V,H,W) and, with a feature head, feat
    (V,16,H,W). check=True sizes the render context for the new poses (one
    synchronising count pass); check=False trusts the current capacity.
    """
    rgb, depth, alpha, fimg = _DecodeRender.apply(xi, xyz, feat, off, params, tr, check)
    out = {"rgb": rgb, "depth": depth, "alpha": alpha}
    if tr.r.a.n_feat:
        out["feat"] = fimg
    return out


def _raise_on_overflow(rc: RenderContext):
    """An overflowed forward renders incomplete images and its backward gives
    zero gradients: refuse to return them (one synchronising header read)."""
    ni, _, ov = rc.status()
    if ov:
        raise RuntimeError(f"render context overflow: {ni} intersections exceed the capacity {rc.capacity}; "
                           "render with check=True or enlarge the context")


class GaussianRenderer:
    """Render context for plain (explicit) Gaussians seen by a fixed set of
    cameras of one resolution, whose poses are base poses times a twist as in
    TrackedRenderer."""

    def __init__(self, cams: Sequence, n_gauss: int, n_feat: int = 0, **opt_kw):
        self.base = [T_cw_of(c) for c in cams]
        self.intr = list(cams)
        self.rc = RenderContext(self.intr, n_gauss, n_feat=n_feat, **opt_kw)
        self.n, self.nf = int(n_gauss), int(n_feat)
        self.generation = 0

    @property
    def V(self) -> int:
        return len(self.base)

    def place(self, xi: Optional[np.ndarray]):
        if xi is None:
            cams = self.intr
        else:
            cams = [camera_at(c, se3_exp(xi[v]) @ self.base[v]) for v, c in enumerate(self.intr)]
        self.rc.set_cameras(cams)


class _RenderGaussians(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, mean, scale, rot, opacity, rgb, feat, gr: GaussianRenderer, check: bool):
        V = gr.V
        xi_h = None if xi is None else xi.detach().to("cpu", torch.float64).numpy().reshape(V, 6)
        gr.place(xi_h)
        g = {"mean": mean.detach().contiguous(), "scale": scale.detach().contiguous(),
             "rot": rot.detach().contiguous(), "opacity": opacity.detach().contiguous(),
             "rgb": rgb.detach().contiguous()}
        if gr.nf:
            g["feat"] = feat.detach().contiguous()
        if check:
            gr.rc.fit(g)
        img = gr.rc.forward(g)
        gr.generation += 1
        ctx.gr, ctx.gen, ctx.g = gr, gr.generation, g
        ctx.pose = xi is not None
        if ctx.pose:
            ctx.J = torch.as_tensor(np.stack([se3_left_jacobian(x) for x in xi_h]), dtype=torch.float32,
                                    device=mean.device)
        ctx.shapes = {k: v.shape for k, v in img.items()}
        return img["rgb"], img["depth"], img["alpha"], img["feat"] if gr.nf else img["depth"].new_zeros(0)

    @staticmethod
    def backward(ctx, d_rgb, d_depth, d_alpha, d_feat):
        gr = ctx.gr
        if gr.generation != ctx.gen:
            raise RuntimeError("GaussianRenderer: backward after a newer forward on the same renderer")
        _raise_on_overflow(gr.rc)

        def g(x, key):
            return x.contiguous() if x is not None else torch.zeros(ctx.shapes[key], device=ctx.g["mean"].device)
        dimg = {"rgb": g(d_rgb, "rgb"), "depth": g(d_depth, "depth"), "alpha": g(d_alpha, "alpha")}
        if gr.nf:
            dimg["feat"] = g(d_feat, "feat")
        dg, d_pose = gr.rc.backward(ctx.g, dimg, pose=ctx.pose)
        d_xi = None
        if ctx.pose:
            d_xi = torch.bmm(ctx.J.transpose(1, 2).contiguous(), d_pose[:, :, None])[:, :, 0]
        # the views share one set of Gaussians: their gradients add up
        red = {k: v.sum(0) for k, v in dg.items()}
        return (d_xi, red["mean"], red["scale"], red["rot"], red["opacity"], red["rgb"],
                red.get("feat"), None, None)


def render_gaussians(mean: torch.Tensor, log_scale: torch.Tensor, rot: torch.Tensor, logit_opacity: torch.Tensor,
                     rgb: torch.Tensor, gr: GaussianRenderer, feat: Optional[torch.Tensor] = None,
                     xi: Optional[torch.Tensor] = None, check: bool = True) -> Dict[str, torch.Tensor]:
    """Differentiable render of plain Gaussians (Sec. 3.1, Eq. 2, Eq. 3) with
    the usual 3DGS parametrisation: scale = exp(log_scale), opacity =
    sigmoid(logit_opacity), quaternion rot (any norm). Planes [c][n] float32
    on the device. With xi ((V, 6) twists), the views are rendered at
    Exp(xi_v) T_cw,v and xi receives its gradient. Returns rgb (V,3,H,W),
    depth, alpha (V,H,W) and, with features, feat (V,16,H,W)."""
    scale = torch.exp(log_scale)
    opacity = torch.sigmoid(logit_opacity)
    rgb_, depth, alpha, fimg = _RenderGaussians.apply(xi, mean, scale, rot, opacity, rgb, feat, gr, check)
    out = {"rgb": rgb_, "depth": depth, "alpha": alpha}
    if gr.nf:
        out["feat"] = fimg
    return out
