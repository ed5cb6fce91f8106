"""Tensor-level wrappers over the C ABI: device buffers, contexts, packing.

Torch is used for device memory and streams only; every step of the path runs
in libasgs kernels.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import torch

from . import _lib as L

HEADS = (("opacity", 1), ("rgb", 3), ("scale", 3), ("rot", 4), ("feat", 16))


def _dev(x, device="cuda"):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float32).contiguous()
    return torch.as_tensor(x, dtype=torch.float32, device=device).contiguous()


def gaussians_to_device(planes: Dict[str, object], device="cuda") -> Dict[str, torch.Tensor]:
    """[c][n] float arrays (numpy or tensors) -> contiguous float32 device tensors."""
    return {k: _dev(v, device) for k, v in planes.items() if v is not None}


def pack_params(weights: Dict[str, Dict[str, object]], k: int, n_feat: int = 16, device="cuda") -> torch.Tensor:
    """Head weights {head: {W1, b1, W2, b2}} -> the packed parameter vector of
    the decoder ABI (per head in order opacity, rgb, scale, rot, feat: the
    first 35 columns of W1 row-major, b1, W2 row-major, b2, then W1's other
    in_dim - 35 columns row-major)."""
    parts = []
    for name, m in HEADS:
        if name == "feat" and n_feat == 0:
            continue
        w = weights[name]
        W1 = _dev(w["W1"], device)
        parts.append(W1[:, :35].reshape(-1))
        for key in ("b1", "W2", "b2"):
            parts.append(_dev(w[key], device).reshape(-1))
        parts.append(W1[:, 35:].reshape(-1))
    return torch.cat(parts)


def unpack_params(flat: torch.Tensor, k: int, n_feat: int = 16, in_dim: int = 35) -> Dict[str, Dict[str, torch.Tensor]]:
    """Inverse of pack_params: {head: {W1 (32, in_dim), b1, W2, b2}}."""
    out, o = {}, 0
    nx = in_dim - 35
    for name, m in HEADS:
        if name == "feat":
            if n_feat == 0:
                continue
            m = n_feat
        shapes = dict(W1=(32, 35), b1=(32,), W2=(k * m, 32), b2=(k * m,), W1x=(32, nx))
        part = {}
        for key in ("W1", "b1", "W2", "b2", "W1x"):
            sz = 1
            for d in shapes[key]:
                sz *= d
            part[key] = flat[o:o + sz].reshape(shapes[key])
            o += sz
        W1x = part.pop("W1x")
        if nx:
            part["W1"] = torch.cat([part["W1"], W1x], 1)
        out[name] = part
    return out


class RenderContext:
    """Caller-owned context of the render path for a fixed set of cameras
    (one resolution) and Gaussian count. Grows its device buffer when the
    intersection count needs it."""

    def __init__(self, cams: Sequence, n_gauss: int, n_feat: int = 16, capacity: int = 0,
                 device="cuda", **opt_kw):
        self.cams = list(cams)
        self.V = len(self.cams)
        self.H, self.W = int(self.cams[0].height), int(self.cams[0].width)
        for c in self.cams:
            if int(c.height) != self.H or int(c.width) != self.W:
                raise ValueError("RenderContext needs one resolution for all views")
        self.n = int(n_gauss)
        self.nf = int(n_feat)
        self.opts = L.make_opts(n_feat, **opt_kw)
        self.device = device
        self.ctx = None
        self.capacity = 0
        self.ensure(max(int(capacity), 1))

    def set_cameras(self, cams: Sequence):
        cams = list(cams)
        if len(cams) != self.V:
            raise ValueError("number of views is fixed per context")
        self.cams = cams

    def ensure(self, capacity: int):
        if capacity <= self.capacity and self.ctx is not None:
            return
        nbytes = L.render_ctx_size(self.cams, self.n, self.opts, int(capacity))
        self.ctx = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.capacity = int(capacity)

    def count(self, g: Dict[str, torch.Tensor]) -> int:
        return L.render_count(self.cams, L.make_gaussians(g, self.n), self.opts, self.ctx)

    def fit(self, g: Dict[str, torch.Tensor], slack: float = 1.25) -> int:
        """Size the context for g (one synchronising count pass)."""
        need = self.count(g)
        if need > self.capacity:
            self.ensure(int(need * slack) + 1024)
        return need

    def new_images(self) -> Dict[str, torch.Tensor]:
        V, H, W = self.V, self.H, self.W
        kw = dict(dtype=torch.float32, device=self.device)
        img = dict(rgb=torch.empty((V, 3, H, W), **kw), depth=torch.empty((V, H, W), **kw),
                   alpha=torch.empty((V, H, W), **kw))
        if self.nf:
            img["feat"] = torch.empty((V, self.nf, H, W), **kw)
        return img

    def forward(self, g: Dict[str, torch.Tensor], out: Optional[Dict[str, torch.Tensor]] = None):
        out = out if out is not None else self.new_images()
        L.render_forward(self.cams, L.make_gaussians(g, self.n), self.opts, L.make_images(out), self.ctx)
        return out

    def forward_l1(self, g: Dict[str, torch.Tensor], targets: Dict[str, torch.Tensor],
                   grad: Dict[str, torch.Tensor], scale: Dict[str, float], weight: Optional[torch.Tensor] = None,
                   loss: Optional[torch.Tensor] = None, out: Optional[Dict[str, torch.Tensor]] = None):
        """Forward render and the weighted L1 residual gradient (and, with
        loss, the per-view loss) in one pass (asgs_render_forward_l1): the
        images and grad as render_forward followed by l1_loss_grad."""
        out = out if out is not None else self.new_images()
        L.render_forward_l1(self.cams, L.make_gaussians(g, self.n), self.opts, L.make_images(out),
                            l1_targets(targets, scale, weight), L.make_images(grad), loss, self.ctx)
        return out

    def new_grads(self) -> Dict[str, torch.Tensor]:
        V, n = self.V, self.n
        kw = dict(dtype=torch.float32, device=self.device)
        dg = dict(mean=torch.empty((V, 3, n), **kw), scale=torch.empty((V, 3, n), **kw),
                  rot=torch.empty((V, 4, n), **kw), opacity=torch.empty((V, n), **kw),
                  rgb=torch.empty((V, 3, n), **kw))
        if self.nf:
            dg["feat"] = torch.empty((V, self.nf, n), **kw)
        return dg

    def backward(self, g: Dict[str, torch.Tensor], dimg: Dict[str, torch.Tensor], pose: bool = True,
                 dg: Optional[Dict[str, torch.Tensor]] = None):
        dg = dg if dg is not None else self.new_grads()
        d_pose = torch.empty((self.V, 6), dtype=torch.float32, device=self.device) if pose else None
        L.render_backward(self.cams, L.make_gaussians(g, self.n), self.opts, L.make_images(dimg),
                          L.make_gaussians(dg, self.n), d_pose, self.ctx)
        return dg, d_pose

    def status(self):
        return L.ctx_status(self.ctx)

    def array(self, which: int, dtype, count: Optional[int] = None, width: int = 1) -> torch.Tensor:
        """Copy of an internal context array (see asgs_ctx_array)."""
        ptr, n = L.ctx_array(self.cams, self.n, self.opts, self.ctx, which)
        if count is not None:
            n = count
        itemsize = torch.empty((), dtype=dtype).element_size()
        base = self.ctx.data_ptr()
        off = ptr - base
        raw = self.ctx[off:off + n * width * itemsize]
        return raw.view(dtype).reshape(n, width) if width > 1 else raw.view(dtype).clone()


class Decoder:
    """Device-resident decoder parameters plus its workspace."""

    def __init__(self, n_anchors: int, k: int, n_feat: int = 16, precision: int = 0, l_o: float = 1.0,
                 l_s: float = 0.02, device="cuda", in_dim: int = 35):
        self.desc = L.make_decoder(n_anchors, k, n_feat, precision, l_o, l_s, in_dim)
        self.in_dim = in_dim
        self.A, self.k, self.nf = n_anchors, k, n_feat
        self.n = n_anchors * k
        self.n_params = L.decode_param_count(self.desc)
        self.device = device
        self.work = None
        self.work_views = 0

    def set_precision(self, precision: int):
        self.desc.precision = precision

    def decode(self, xyz, feat, off, params, cams, out: Optional[Dict[str, torch.Tensor]] = None):
        V = len(cams)
        kw = dict(dtype=torch.float32, device=self.device)
        if out is None:
            out = dict(mean=torch.empty((3, self.n), **kw), scale=torch.empty((V, 3, self.n), **kw),
                       rot=torch.empty((V, 4, self.n), **kw), opacity=torch.empty((V, self.n), **kw),
                       rgb=torch.empty((V, 3, self.n), **kw))
            if self.nf:
                out["feat"] = torch.empty((V, self.nf, self.n), **kw)
        L.decode(self.desc, xyz, feat, off, params, cams, L.make_gaussians(out, self.n))
        return out

    def backward(self, xyz, feat, off, params, cams, dg: Dict[str, torch.Tensor], d_pose=None):
        V = len(cams)
        need = L.decode_workspace_size(self.desc, V)
        if self.work is None or self.work.numel() < need:
            self.work = torch.empty(need, dtype=torch.uint8, device=self.device)
        kw = dict(dtype=torch.float32, device=self.device)
        d_xyz = torch.empty((3, self.A), **kw)
        d_feat = torch.empty((self.A, 32), **kw)
        d_off = torch.empty((3, self.n), **kw)
        d_params = torch.empty((self.n_params,), **kw)
        L.decode_backward(self.desc, xyz, feat, off, params, cams, L.make_gaussians(dg, self.n), d_xyz, d_feat,
                          d_off, d_params, d_pose, self.work)
        return d_xyz, d_feat, d_off, d_params


def l1_targets(targets: Dict[str, torch.Tensor], scale: Dict[str, float],
               weight: Optional[torch.Tensor] = None) -> "L.L1Targets":
    t = L.L1Targets()
    for k in ("rgb", "depth", "feat", "alpha"):
        setattr(t, k, L._ptr(targets.get(k)))
    t.weight = L._ptr(weight)
    for i, k in enumerate(("rgb", "depth", "feat", "alpha")):
        t.scale[i] = float(scale.get(k, 0.0))
    return t


def l1_loss_grad(maps: Dict[str, torch.Tensor], targets: Dict[str, torch.Tensor], grad: Dict[str, torch.Tensor],
                 scale: Dict[str, float], weight: Optional[torch.Tensor] = None,
                 loss: Optional[torch.Tensor] = None) -> Optional[torch.Tensor]:
    """Weighted L1 residual of packed maps (V, C, H, W) against targets in
    one library kernel (asgs_l1_loss): writes sign gradients times scale into
    grad and, with loss (a (V,) tensor), the per-view loss."""
    rgb = maps["rgb"]
    V, H, W = rgb.shape[0], rgb.shape[-2], rgb.shape[-1]
    nf = maps["feat"].shape[1] if "feat" in maps else 0
    t = l1_targets(targets, scale, weight)
    work = None
    if loss is not None:
        work = torch.empty(L.l1_loss_work_size(V), dtype=torch.uint8, device=rgb.device)
    L.l1_loss(V, W, H, nf, L.make_images(maps), t, L.make_images(grad), loss, work)
    return loss


def tracking_residual(rendered: Dict[str, torch.Tensor], cosine: torch.Tensor, obs_rgb: torch.Tensor,
                      obs_depth: torch.Tensor, want_xi: bool = True, **opt_kw) -> Dict[str, torch.Tensor]:
    """Multi-modal residual R (Eq. 6), per-pixel uncertainty sigma and motion
    mask (Eq. 15) and the per-view objective xi, in one library kernel
    (asgs_tracking_residual). rendered: rgb (V,3,H,W), depth, alpha (V,H,W);
    cosine (V,H,W); observations obs_rgb (V,3,H,W), obs_depth (V,H,W)."""
    rgb = rendered["rgb"]
    V, H, W = rgb.shape[0], rgb.shape[-2], rgb.shape[-1]
    dev = rgb.device
    m = L.ResidualMaps()
    c = lambda t: t.contiguous()
    keep = [c(rgb), c(rendered["depth"]), c(rendered["alpha"]), c(cosine), c(obs_rgb), c(obs_depth)]
    m.rgb, m.depth, m.alpha, m.cosine, m.obs_rgb, m.obs_depth = (t.data_ptr() for t in keep)
    out = dict(R=torch.empty((V, H, W), dtype=torch.float32, device=dev),
               sigma=torch.empty((V, H, W), dtype=torch.float32, device=dev),
               dynamic=torch.empty((V, H, W), dtype=torch.uint8, device=dev))
    work = None
    if want_xi:
        out["xi"] = torch.empty(V, dtype=torch.float32, device=dev)
        work = torch.empty(L.residual_work_size(V, W, H), dtype=torch.uint8, device=dev)
    L.tracking_residual(V, W, H, L.residual_opts(**opt_kw), m, out["R"], out["sigma"], out["dynamic"],
                        out.get("xi"), work)
    return out


class FeatureLift:
    """The feature lift F_m and the cosine distillation (asgs_feature_forward
    / asgs_feature_backward) for views of one resolution, with its device
    workspace. params: packed W1 [128][16], b1, W2 [n_high][128], b2."""

    def __init__(self, n_views: int, width: int, height: int, n_high: int, grid_h: int, grid_w: int,
                 device="cuda"):
        self.desc = L.feature_lift(n_high, grid_h, grid_w)
        self.V, self.W, self.H = n_views, width, height
        self.n_params = L.feature_param_count(self.desc)
        self.work = torch.empty(L.feature_workspace_size(self.desc, n_views, width, height), dtype=torch.uint8,
                                device=device)
        self.device = device

    def forward(self, feat: torch.Tensor, params: torch.Tensor, dino: torch.Tensor, want_loss: bool = True):
        """feat (V,16,H,W), dino (V,n_high,grid_h,grid_w) -> cosine (V,H,W), loss (V,) mean 1 - cos."""
        cos = torch.empty((self.V, self.H, self.W), dtype=torch.float32, device=self.device)
        loss = torch.empty(self.V, dtype=torch.float32, device=self.device) if want_loss else None
        L.feature_forward(self.desc, self.V, self.W, self.H, feat.contiguous(), params.contiguous(),
                          dino.contiguous(), cos, loss, self.work)
        return cos, loss

    def backward(self, feat: torch.Tensor, params: torch.Tensor, dino: torch.Tensor, d_cos: torch.Tensor):
        """dL/dcos (V,H,W) -> dL/dfeat (V,16,H,W), dL/dparams (packed)."""
        d_feat = torch.empty((self.V, 16, self.H, self.W), dtype=torch.float32, device=self.device)
        d_params = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        L.feature_backward(self.desc, self.V, self.W, self.H, feat.contiguous(), params.contiguous(),
                           dino.contiguous(), d_cos.contiguous(), d_feat, d_params, self.work)
        return d_feat, d_params


def mapping_loss(rendered: Dict[str, torch.Tensor], obs_rgb: torch.Tensor, obs_depth: torch.Tensor,
                 cosine: Optional[torch.Tensor] = None, dynamic: Optional[torch.Tensor] = None,
                 want_grad: bool = True, **opt_kw) -> Dict[str, torch.Tensor]:
    """Mapping loss of Eq. 4 / Eq. 14 per view with SSIM, and its gradients
    w.r.t. the rendered colour and depth and the distillation cosine, in the
    library's stencil kernels (asgs_mapping_loss). rendered: rgb (V,3,H,W),
    depth (V,H,W); obs_rgb, obs_depth alike; cosine (V,H,W) or None; dynamic
    (V,H,W) uint8 motion mask or None."""
    rgb = rendered["rgb"]
    V, H, W = rgb.shape[0], rgb.shape[-2], rgb.shape[-1]
    dev = rgb.device
    c = lambda t: None if t is None else t.contiguous()
    keep = [c(rgb), c(rendered["depth"]), c(obs_rgb), c(obs_depth), c(cosine), c(dynamic)]
    m = L.MappingMaps()
    m.rgb, m.depth, m.obs_rgb, m.obs_depth, m.cosine, m.dynamic = (L._ptr(t) for t in keep)
    kw = dict(dtype=torch.float32, device=dev)
    out = dict(loss=torch.empty(V, **kw))
    if want_grad:
        out["d_rgb"] = torch.empty((V, 3, H, W), **kw)
        out["d_depth"] = torch.empty((V, H, W), **kw)
        if cosine is not None:
            out["d_cos"] = torch.empty((V, H, W), **kw)
    work = torch.empty(L.mapping_work_size(V, W, H), dtype=torch.uint8, device=dev)
    L.mapping_loss(V, W, H, L.mapping_opts(**opt_kw), m, out["loss"], out.get("d_rgb"), out.get("d_depth"),
                   out.get("d_cos"), work)
    return out


def mean_scale(scale: torch.Tensor, lam5: float = 0.01, d_scale: Optional[torch.Tensor] = None) -> torch.Tensor:
    """s_bar of Eq. 14 (device scalar); adds lam5 / count to d_scale if given."""
    value = torch.empty(1, dtype=torch.float32, device=scale.device)
    work = torch.empty(L.mean_scale_work_size(), dtype=torch.uint8, device=scale.device)
    L.mean_scale(scale.contiguous(), lam5, value, d_scale, work)
    return value


class UncertaintyMLP:
    """The uncertainty MLP F_u with its loss L_u and the motion mask
    (asgs_uncertainty) for views of one resolution, with its device
    workspace. params: packed W1 [128][n_high], b1, w2 [128], b2."""

    def __init__(self, n_views: int, width: int, height: int, n_high: int, grid_h: int, grid_w: int,
                 sigma_min: float = 1e-3, lam3: float = 0.4, device="cuda"):
        self.desc = L.uncertainty_mlp(n_high, grid_h, grid_w, sigma_min, lam3)
        self.V, self.W, self.H = n_views, width, height
        self.n_params = L.uncertainty_param_count(self.desc)
        self.work = torch.empty(L.uncertainty_workspace_size(self.desc, n_views, width, height), dtype=torch.uint8,
                                device=device)
        self.device = device

    def __call__(self, params: torch.Tensor, dino: torch.Tensor, R: Optional[torch.Tensor] = None,
                 want_grad: bool = True) -> Dict[str, torch.Tensor]:
        """dino (V,n_high,grid_h,grid_w), R (V,H,W) or None -> sigma, dynamic
        (V,H,W); with R also loss (V,) and, with want_grad, d_params."""
        kw = dict(dtype=torch.float32, device=self.device)
        out = dict(sigma=torch.empty((self.V, self.H, self.W), **kw),
                   dynamic=torch.empty((self.V, self.H, self.W), dtype=torch.uint8, device=self.device))
        if R is not None:
            out["loss"] = torch.empty(self.V, **kw)
            if want_grad:
                out["d_params"] = torch.empty(self.n_params, **kw)
        L.uncertainty(self.desc, self.V, self.W, self.H, params.contiguous(), dino.contiguous(),
                      None if R is None else R.contiguous(), out["sigma"], out["dynamic"], out.get("loss"),
                      out.get("d_params"), self.work)
        return out
