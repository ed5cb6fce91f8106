"""Anchor scene -> decode -> render, and the backward to anchors, head-MLP
parameters and camera poses, on device (all steps in libasgs kernels)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from .core import Decoder, RenderContext, pack_params


@dataclass
class DeviceAnchors:
    xyz: torch.Tensor      # (3, A)
    feat: torch.Tensor     # (A, 32)
    off: torch.Tensor      # (3, A*k)
    params: torch.Tensor   # packed head parameters
    k: int
    n_feat: int
    l_o: float
    l_s: float
    in_dim: int = 35

    @property
    def A(self) -> int:
        return int(self.xyz.shape[1])


def anchors_to_device(scene, device="cuda") -> DeviceAnchors:
    """From an object with xyz (3,A), feat (A,32), off (3,A*k), k, weights
    {head: {W1,b1,W2,b2}}, l_o, l_s (numpy or tensors)."""
    nf = 16 if "feat" in scene.weights else 0

    def t(x):
        return torch.as_tensor(x, dtype=torch.float32).to(device).contiguous()
    return DeviceAnchors(xyz=t(scene.xyz), feat=t(scene.feat), off=t(scene.off),
                         params=pack_params(scene.weights, scene.k, nf, device), k=int(scene.k),
                         n_feat=nf, l_o=float(scene.l_o), l_s=float(scene.l_s),
                         in_dim=int(np.shape(scene.weights["opacity"]["W1"])[1]))


class AnchorRenderer:
    """Decode + render for a batch of views of one resolution."""

    def __init__(self, anchors: DeviceAnchors, cams: Sequence, precision: int = 0, capacity: int = 0,
                 **opt_kw):
        self.a = anchors
        self.cams = list(cams)
        self.dec = Decoder(anchors.A, anchors.k, anchors.n_feat, precision, anchors.l_o, anchors.l_s,
                           in_dim=anchors.in_dim)
        self.rc = RenderContext(self.cams, anchors.A * anchors.k, anchors.n_feat, capacity, **opt_kw)
        self.g = None
        self.images = None
        self.dg = None

    def set_cameras(self, cams: Sequence):
        self.cams = list(cams)
        self.rc.set_cameras(self.cams)

    def decode(self):
        a = self.a
        self.g = self.dec.decode(a.xyz, a.feat, a.off, a.params, self.cams, out=self.g)
        return self.g

    def fit(self, slack: float = 1.25) -> int:
        """Decode and size the render context exactly (synchronises)."""
        self.decode()
        return self.rc.fit(self.g, slack)

    def forward(self) -> Dict[str, torch.Tensor]:
        self.decode()
        self.images = self.rc.forward(self.g, out=self.images)
        return self.images

    def forward_l1(self, targets: Dict[str, torch.Tensor], grad: Dict[str, torch.Tensor], scale: Dict[str, float],
                   weight: Optional[torch.Tensor] = None, loss: Optional[torch.Tensor] = None):
        """Decode, render and the weighted L1 residual gradient in the
        forward's output stage (RenderContext.forward_l1)."""
        self.decode()
        self.images = self.rc.forward_l1(self.g, targets, grad, scale, weight, loss, out=self.images)
        return self.images

    def backward(self, dimg: Dict[str, torch.Tensor], pose: bool = True, render_only: bool = False):
        """dimg: upstream gradients shaped like the images. Returns dict with
        d_gauss (per view) and, unless render_only, d_xyz, d_feat, d_off,
        d_params, and d_pose (V,6) including the decoder's camera-centre term."""
        a = self.a
        self.dg, d_pose = self.rc.backward(self.g, dimg, pose=pose, dg=self.dg)
        out = dict(d_gauss=self.dg, d_pose=d_pose)
        if render_only:
            return out
        d_xyz, d_feat, d_off, d_params = self.dec.backward(a.xyz, a.feat, a.off, a.params, self.cams, self.dg,
                                                           d_pose=d_pose)
        out.update(d_xyz=d_xyz, d_feat=d_feat, d_off=d_off, d_params=d_params)
        return out
