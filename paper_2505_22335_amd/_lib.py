"""ctypes binding of libasgs (include/asgs.h): argument marshalling only.

Every array is a torch tensor on the GPU (float32 unless stated); the binding
passes its data pointer and the current HIP stream and checks the returned
status. If the library is missing this module raises on import: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Dict, Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libasgs.so")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
HEADERS = [os.path.join(INCLUDE, h) for h in ("asgs.h", "asgs_serve.h")]

# torch ships its own HIP runtime under the same soname as the system one; it
# must be the first loaded so that torch's allocations and this library share
# one runtime (otherwise whichever loads second sees no device).
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libasgs.so not built at {LIB_PATH}: run python paper_2505_22335_amd/build.py")
lib = C.CDLL(LIB_PATH)

OK, E_INVALID, E_WORKSPACE, E_CAPACITY, E_DEVICE, E_UNSUPPORTED = range(6)
MAX_VIEWS = 64
(K_PROJECT, K_SORT, K_BLEND_FWD, K_BLEND_BWD, K_PROJECT_BWD, K_DECODE, K_DECODE_BWD, K_RESIDUAL, K_FEATURE,
 K_FEATURE_BWD, K_MAPPING, K_UNCERTAINTY) = range(12)
K_NUM = 12
(CTX_PAIR_TILE, CTX_PAIR_GAUSS, CTX_TILE_RANGE, CTX_RECT, CTX_NCONTRIB, CTX_TFINAL, CTX_GEOM, CTX_RADIUS,
 CTX_DEPTH_KEY, CTX_NTILES) = range(1, 11)


class AsgsError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.asgs_last_error().decode()
        super().__init__(f"{where}: {lib.asgs_status_string(status).decode()} ({status}): {msg}")
        self.status = status


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("T_wc", C.c_float * 12), ("t", C.c_float)]


class RenderOpts(C.Structure):
    _fields_ = [("tile", C.c_int32), ("n_feat", C.c_int32), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("T_min", C.c_float), ("dilation", C.c_float),
                ("znear", C.c_float), ("fov_clamp", C.c_float), ("bg", C.c_float * 3),
                ("extent_mode", C.c_int32)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("rot", C.c_void_p),
                ("opacity", C.c_void_p), ("rgb", C.c_void_p), ("feat", C.c_void_p),
                ("view_stride", C.c_int64 * 6)]


class Images(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("feat", C.c_void_p), ("alpha", C.c_void_p)]


class Decoder(C.Structure):
    _fields_ = [("n_anchors", C.c_int64), ("k", C.c_int32), ("n_feat", C.c_int32),
                ("precision", C.c_int32), ("l_o", C.c_float), ("l_s", C.c_float),
                ("in_dim", C.c_int32)]


class L1Targets(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("feat", C.c_void_p), ("alpha", C.c_void_p),
                ("weight", C.c_void_p), ("scale", C.c_float * 4)]


class ResidualOpts(C.Structure):
    _fields_ = [("w_rgb", C.c_float), ("w_depth", C.c_float), ("w_feat", C.c_float), ("vis_T", C.c_float),
                ("sigma_min", C.c_float), ("dyn_thresh", C.c_float), ("reserved", C.c_int32)]


class ResidualMaps(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p), ("cosine", C.c_void_p),
                ("obs_rgb", C.c_void_p), ("obs_depth", C.c_void_p)]


class FeatureLift(C.Structure):
    _fields_ = [("n_high", C.c_int32), ("grid_h", C.c_int32), ("grid_w", C.c_int32), ("reserved", C.c_int32)]


class AnchorUpdateOpts(C.Structure):
    _fields_ = [("prior", C.c_float), ("p_min", C.c_float), ("p_max", C.c_float), ("prune_below", C.c_float),
                ("reserved", C.c_int32)]


class MappingOpts(C.Structure):
    _fields_ = [("lam", C.c_float), ("lam1", C.c_float), ("lam2", C.c_float), ("lam4", C.c_float),
                ("reserved", C.c_int32)]


class MappingMaps(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("obs_rgb", C.c_void_p), ("obs_depth", C.c_void_p),
                ("cosine", C.c_void_p), ("dynamic", C.c_void_p)]


class UncertaintyMlp(C.Structure):
    _fields_ = [("n_high", C.c_int32), ("grid_h", C.c_int32), ("grid_w", C.c_int32), ("sigma_min", C.c_float),
                ("lam3", C.c_float), ("reserved", C.c_int32)]


P = C.c_void_p
_sigs = {
    "asgs_abi_version": (C.c_int, []),
    "asgs_status_string": (C.c_char_p, [C.c_int]),
    "asgs_last_error": (C.c_char_p, []),
    "asgs_render_opts_default": (None, [C.POINTER(RenderOpts)]),
    "asgs_render_ctx_size": (C.c_int, [C.POINTER(Camera), C.c_int32, C.c_int64, C.POINTER(RenderOpts),
                                       C.c_int64, C.POINTER(C.c_size_t)]),
    "asgs_render_count": (C.c_int, [C.POINTER(Camera), C.c_int32, C.POINTER(Gaussians), C.POINTER(RenderOpts),
                                    P, C.c_size_t, C.POINTER(C.c_int64), P]),
    "asgs_render_forward": (C.c_int, [C.POINTER(Camera), C.c_int32, C.POINTER(Gaussians),
                                      C.POINTER(RenderOpts), C.POINTER(Images), P, C.c_size_t, P]),
    "asgs_render_forward_l1": (C.c_int, [C.POINTER(Camera), C.c_int32, C.POINTER(Gaussians),
                                         C.POINTER(RenderOpts), C.POINTER(Images), C.POINTER(L1Targets),
                                         C.POINTER(Images), P, P, C.c_size_t, P]),
    "asgs_render_backward": (C.c_int, [C.POINTER(Camera), C.c_int32, C.POINTER(Gaussians),
                                       C.POINTER(RenderOpts), C.POINTER(Images), C.POINTER(Gaussians), P, P,
                                       C.c_size_t, P]),
    "asgs_ctx_status": (C.c_int, [P, P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "asgs_ctx_array": (C.c_int, [C.POINTER(Camera), C.c_int32, C.c_int64, C.POINTER(RenderOpts), P,
                                 C.c_size_t, C.c_int32, C.POINTER(P), C.POINTER(C.c_int64)]),
    "asgs_decode_param_count": (C.c_int, [C.POINTER(Decoder), C.POINTER(C.c_int64)]),
    "asgs_decode": (C.c_int, [C.POINTER(Decoder), P, P, P, P, C.POINTER(Camera), C.c_int32,
                              C.POINTER(Gaussians), P]),
    "asgs_decode_workspace_size": (C.c_int, [C.POINTER(Decoder), C.c_int32, C.POINTER(C.c_size_t)]),
    "asgs_decode_backward": (C.c_int, [C.POINTER(Decoder), P, P, P, P, C.POINTER(Camera), C.c_int32,
                                       C.POINTER(Gaussians), P, P, P, P, P, P, C.c_size_t, P]),
    "asgs_l1_loss_work_size": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "asgs_l1_loss": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Images), C.POINTER(L1Targets),
                               C.POINTER(Images), P, P, C.c_size_t, P]),
    "asgs_l1_loss_noalloc": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(Images),
                                       C.POINTER(L1Targets), C.POINTER(Images), P, P]),
    "asgs_residual_opts_default": (None, [C.POINTER(ResidualOpts)]),
    "asgs_residual_work_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "asgs_tracking_residual": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(ResidualOpts),
                                         C.POINTER(ResidualMaps), P, P, P, P, P, C.c_size_t, P]),
    "asgs_feature_param_count": (C.c_int, [C.POINTER(FeatureLift), C.POINTER(C.c_int64)]),
    "asgs_feature_workspace_size": (C.c_int, [C.POINTER(FeatureLift), C.c_int32, C.c_int32, C.c_int32,
                                              C.POINTER(C.c_size_t)]),
    "asgs_feature_forward": (C.c_int, [C.POINTER(FeatureLift), C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P,
                                       C.c_size_t, P]),
    "asgs_feature_backward": (C.c_int, [C.POINTER(FeatureLift), C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P,
                                        P, C.c_size_t, P]),
    "asgs_anchor_update": (C.c_int, [C.c_int64, C.POINTER(AnchorUpdateOpts), P, P, P, P, P]),
    "asgs_mapping_opts_default": (None, [C.POINTER(MappingOpts)]),
    "asgs_mapping_work_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "asgs_mapping_loss": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(MappingOpts), C.POINTER(MappingMaps),
                                    P, P, P, P, P, C.c_size_t, P]),
    "asgs_mean_scale_work_size": (C.c_int, [C.POINTER(C.c_size_t)]),
    "asgs_uncertainty_param_count": (C.c_int, [C.POINTER(UncertaintyMlp), C.POINTER(C.c_int64)]),
    "asgs_uncertainty_workspace_size": (C.c_int, [C.POINTER(UncertaintyMlp), C.c_int32, C.c_int32, C.c_int32,
                                                  C.POINTER(C.c_size_t)]),
    "asgs_uncertainty": (C.c_int, [C.POINTER(UncertaintyMlp), C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P,
                                   P, C.c_size_t, P]),
    "asgs_mean_scale": (C.c_int, [C.c_int64, P, C.c_float, P, P, P, C.c_size_t, P]),
    "asgs_profile_enable": (C.c_int, [C.c_uint32]),
    "asgs_profile_read": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def declared_functions() -> list:
    """Function names declared in the public headers (include/*.h)."""
    names = set()
    for h in HEADERS:
        with open(h) as f:
            txt = f.read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(asgs_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def check(status: int, where: str):
    if status != OK:
        raise AsgsError(status, where)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---------------------------------------------------------------------------
# Struct builders
# ---------------------------------------------------------------------------

def make_cameras(cams: Sequence) -> "C.Array":
    """Objects with width, height, fx, fy, cx, cy, T_wc (3x4) and optionally
    t (frame time, default 0) -> Camera[]."""
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].width, arr[i].height = int(c.width), int(c.height)
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        T = [float(x) for row in c.T_wc for x in row]
        for k in range(12):
            arr[i].T_wc[k] = T[k]
        arr[i].t = float(getattr(c, "t", 0.0))
    return arr


def make_opts(n_feat: int = 16, **kw) -> RenderOpts:
    o = RenderOpts()
    lib.asgs_render_opts_default(C.byref(o))
    o.n_feat = n_feat
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = float(v[i])
        else:
            setattr(o, k, v)
    return o


FIELDS = ("mean", "scale", "rot", "opacity", "rgb", "feat")


def make_gaussians(g: Dict[str, "object"], n: int) -> Gaussians:
    """g maps field -> tensor of shape [c][n] (one view) or [V][c][n] (per
    view). A 2D/1D tensor is shared by every view (stride 0)."""
    s = Gaussians()
    s.n = n
    for i, f in enumerate(FIELDS):
        t = g.get(f)
        if t is None:
            setattr(s, f, None)
            s.view_stride[i] = 0
            continue
        per_view = (t.dim() == 3) or (f == "opacity" and t.dim() == 2)
        setattr(s, f, t.data_ptr())
        s.view_stride[i] = t[0].numel() if per_view else 0
    return s


def make_images(img: Dict[str, "object"]) -> Images:
    s = Images()
    s.rgb, s.depth, s.feat, s.alpha = (_ptr(img.get(k)) for k in ("rgb", "depth", "feat", "alpha"))
    return s


# ---------------------------------------------------------------------------
# Calls
# ---------------------------------------------------------------------------

def render_ctx_size(cams, n_gauss: int, opts: RenderOpts, capacity: int) -> int:
    b = C.c_size_t()
    ca = make_cameras(cams)
    check(lib.asgs_render_ctx_size(ca, len(cams), n_gauss, C.byref(opts), capacity, C.byref(b)),
          "asgs_render_ctx_size")
    return b.value


def render_count(cams, g: Gaussians, opts: RenderOpts, ctx, stream=None) -> int:
    n = C.c_int64()
    ca = make_cameras(cams)
    check(lib.asgs_render_count(ca, len(cams), C.byref(g), C.byref(opts), ctx.data_ptr(), ctx.numel(),
                                C.byref(n), _stream(stream)), "asgs_render_count")
    return n.value


def render_forward(cams, g: Gaussians, opts: RenderOpts, out: Images, ctx, stream=None):
    ca = make_cameras(cams)
    check(lib.asgs_render_forward(ca, len(cams), C.byref(g), C.byref(opts), C.byref(out), ctx.data_ptr(),
                                  ctx.numel(), _stream(stream)), "asgs_render_forward")


def render_forward_l1(cams, g: Gaussians, opts: RenderOpts, out: Images, targets: "L1Targets", grad: Images,
                      loss, ctx, stream=None):
    ca = make_cameras(cams)
    check(lib.asgs_render_forward_l1(ca, len(cams), C.byref(g), C.byref(opts), C.byref(out), C.byref(targets),
                                     C.byref(grad), _ptr(loss), ctx.data_ptr(), ctx.numel(), _stream(stream)),
          "asgs_render_forward_l1")


def render_backward(cams, g: Gaussians, opts: RenderOpts, dout: Images, dg: Gaussians, d_pose, ctx,
                    stream=None):
    ca = make_cameras(cams)
    check(lib.asgs_render_backward(ca, len(cams), C.byref(g), C.byref(opts), C.byref(dout), C.byref(dg),
                                   _ptr(d_pose), ctx.data_ptr(), ctx.numel(), _stream(stream)),
          "asgs_render_backward")


def ctx_status(ctx, stream=None):
    ni, nv, ov = C.c_int64(), C.c_int64(), C.c_int32()
    check(lib.asgs_ctx_status(ctx.data_ptr(), _stream(stream), C.byref(ni), C.byref(nv), C.byref(ov)),
          "asgs_ctx_status")
    return ni.value, nv.value, ov.value


def ctx_array(cams, n_gauss: int, opts: RenderOpts, ctx, which: int):
    p, n = C.c_void_p(), C.c_int64()
    ca = make_cameras(cams)
    check(lib.asgs_ctx_array(ca, len(cams), n_gauss, C.byref(opts), ctx.data_ptr(), ctx.numel(), which,
                             C.byref(p), C.byref(n)), "asgs_ctx_array")
    return p.value, n.value


def make_decoder(n_anchors: int, k: int, n_feat: int = 16, precision: int = 0, l_o: float = 1.0,
                 l_s: float = 0.02, in_dim: int = 35) -> Decoder:
    d = Decoder()
    d.n_anchors, d.k, d.n_feat, d.precision, d.l_o, d.l_s = n_anchors, k, n_feat, precision, l_o, l_s
    d.in_dim = in_dim
    return d


def decode_param_count(d: Decoder) -> int:
    n = C.c_int64()
    check(lib.asgs_decode_param_count(C.byref(d), C.byref(n)), "asgs_decode_param_count")
    return n.value


def decode_workspace_size(d: Decoder, n_views: int) -> int:
    b = C.c_size_t()
    check(lib.asgs_decode_workspace_size(C.byref(d), n_views, C.byref(b)), "asgs_decode_workspace_size")
    return b.value


def decode(d: Decoder, xyz, feat, off, params, cams, out: Gaussians, stream=None):
    ca = make_cameras(cams)
    check(lib.asgs_decode(C.byref(d), xyz.data_ptr(), feat.data_ptr(), off.data_ptr(), params.data_ptr(), ca,
                          len(cams), C.byref(out), _stream(stream)), "asgs_decode")


def decode_backward(d: Decoder, xyz, feat, off, params, cams, dg: Gaussians, d_xyz, d_feat, d_off, d_params,
                    d_pose, work, stream=None):
    ca = make_cameras(cams)
    check(lib.asgs_decode_backward(C.byref(d), xyz.data_ptr(), feat.data_ptr(), off.data_ptr(),
                                   params.data_ptr(), ca, len(cams), C.byref(dg), _ptr(d_xyz),
                                   _ptr(d_feat), _ptr(d_off), _ptr(d_params), _ptr(d_pose),
                                   work.data_ptr(), work.numel(), _stream(stream)), "asgs_decode_backward")


def l1_loss_work_size(n_views: int) -> int:
    b = C.c_size_t()
    check(lib.asgs_l1_loss_work_size(n_views, C.byref(b)), "asgs_l1_loss_work_size")
    return b.value


def l1_loss(n_views: int, width: int, height: int, n_feat: int, maps: Images, targets: L1Targets, grad: Images,
            loss=None, work=None, stream=None):
    check(lib.asgs_l1_loss(n_views, width, height, n_feat, C.byref(maps), C.byref(targets), C.byref(grad),
                           _ptr(loss), _ptr(work), 0 if work is None else work.numel(), _stream(stream)),
          "asgs_l1_loss")


def l1_loss_noalloc(n_views: int, width: int, height: int, n_feat: int, maps: Images, targets: L1Targets,
                    grad: Images, loss=None, stream=None):
    check(lib.asgs_l1_loss_noalloc(n_views, width, height, n_feat, C.byref(maps), C.byref(targets), C.byref(grad),
                                   _ptr(loss), _stream(stream)), "asgs_l1_loss_noalloc")


def residual_opts(**kw) -> ResidualOpts:
    o = ResidualOpts()
    lib.asgs_residual_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def residual_work_size(n_views: int, width: int, height: int) -> int:
    b = C.c_size_t()
    check(lib.asgs_residual_work_size(n_views, width, height, C.byref(b)), "asgs_residual_work_size")
    return b.value


def tracking_residual(n_views: int, width: int, height: int, opts: ResidualOpts, maps: ResidualMaps, R=None,
                      sigma=None, dynamic=None, xi=None, work=None, stream=None):
    check(lib.asgs_tracking_residual(n_views, width, height, C.byref(opts), C.byref(maps), _ptr(R), _ptr(sigma),
                                     _ptr(dynamic), _ptr(xi), _ptr(work), 0 if work is None else work.numel(),
                                     _stream(stream)), "asgs_tracking_residual")


def feature_lift(n_high: int, grid_h: int, grid_w: int) -> FeatureLift:
    f = FeatureLift()
    f.n_high, f.grid_h, f.grid_w, f.reserved = n_high, grid_h, grid_w, 0
    return f


def feature_param_count(f: FeatureLift) -> int:
    n = C.c_int64()
    check(lib.asgs_feature_param_count(C.byref(f), C.byref(n)), "asgs_feature_param_count")
    return n.value


def feature_workspace_size(f: FeatureLift, n_views: int, width: int, height: int) -> int:
    b = C.c_size_t()
    check(lib.asgs_feature_workspace_size(C.byref(f), n_views, width, height, C.byref(b)),
          "asgs_feature_workspace_size")
    return b.value


def feature_forward(f: FeatureLift, n_views: int, width: int, height: int, feat, params, dino, cosine, loss, work,
                    stream=None):
    check(lib.asgs_feature_forward(C.byref(f), n_views, width, height, feat.data_ptr(), params.data_ptr(),
                                   dino.data_ptr(), cosine.data_ptr(), _ptr(loss), work.data_ptr(), work.numel(),
                                   _stream(stream)), "asgs_feature_forward")


def feature_backward(f: FeatureLift, n_views: int, width: int, height: int, feat, params, dino, d_cos, d_feat,
                     d_params, work, stream=None):
    check(lib.asgs_feature_backward(C.byref(f), n_views, width, height, feat.data_ptr(), params.data_ptr(),
                                    dino.data_ptr(), d_cos.data_ptr(), d_feat.data_ptr(), d_params.data_ptr(),
                                    work.data_ptr(), work.numel(), _stream(stream)), "asgs_feature_backward")


def anchor_update(p_obs, p, keep=None, n_keep=None, prior=0.5, p_min=0.0, p_max=1.0, prune_below=0.0,
                  stream=None):
    o = AnchorUpdateOpts()
    o.prior, o.p_min, o.p_max, o.prune_below, o.reserved = prior, p_min, p_max, prune_below, 0
    check(lib.asgs_anchor_update(p.numel(), C.byref(o), p_obs.data_ptr(), p.data_ptr(), _ptr(keep), _ptr(n_keep),
                                 _stream(stream)), "asgs_anchor_update")


def mapping_opts(**kw) -> MappingOpts:
    o = MappingOpts()
    lib.asgs_mapping_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mapping_work_size(n_views: int, width: int, height: int) -> int:
    b = C.c_size_t()
    check(lib.asgs_mapping_work_size(n_views, width, height, C.byref(b)), "asgs_mapping_work_size")
    return b.value


def mapping_loss(n_views: int, width: int, height: int, opts: MappingOpts, maps: MappingMaps, loss=None, d_rgb=None,
                 d_depth=None, d_cos=None, work=None, stream=None):
    check(lib.asgs_mapping_loss(n_views, width, height, C.byref(opts), C.byref(maps), _ptr(loss), _ptr(d_rgb),
                                _ptr(d_depth), _ptr(d_cos), _ptr(work), 0 if work is None else work.numel(),
                                _stream(stream)), "asgs_mapping_loss")


def mean_scale_work_size() -> int:
    b = C.c_size_t()
    check(lib.asgs_mean_scale_work_size(C.byref(b)), "asgs_mean_scale_work_size")
    return b.value


def mean_scale(scale, lam5: float, value=None, d_scale=None, work=None, stream=None):
    check(lib.asgs_mean_scale(scale.numel(), scale.data_ptr(), lam5, _ptr(value), _ptr(d_scale), _ptr(work),
                              0 if work is None else work.numel(), _stream(stream)), "asgs_mean_scale")


def uncertainty_mlp(n_high: int, grid_h: int, grid_w: int, sigma_min: float = 1e-3,
                    lam3: float = 0.4) -> UncertaintyMlp:
    u = UncertaintyMlp()
    u.n_high, u.grid_h, u.grid_w, u.sigma_min, u.lam3, u.reserved = n_high, grid_h, grid_w, sigma_min, lam3, 0
    return u


def uncertainty_param_count(u: UncertaintyMlp) -> int:
    n = C.c_int64()
    check(lib.asgs_uncertainty_param_count(C.byref(u), C.byref(n)), "asgs_uncertainty_param_count")
    return n.value


def uncertainty_workspace_size(u: UncertaintyMlp, n_views: int, width: int, height: int) -> int:
    b = C.c_size_t()
    check(lib.asgs_uncertainty_workspace_size(C.byref(u), n_views, width, height, C.byref(b)),
          "asgs_uncertainty_workspace_size")
    return b.value


def uncertainty(u: UncertaintyMlp, n_views: int, width: int, height: int, params, dino, R=None, sigma=None,
                dynamic=None, loss=None, d_params=None, work=None, stream=None):
    check(lib.asgs_uncertainty(C.byref(u), n_views, width, height, params.data_ptr(), dino.data_ptr(), _ptr(R),
                               _ptr(sigma), _ptr(dynamic), _ptr(loss), _ptr(d_params), _ptr(work),
                               0 if work is None else work.numel(), _stream(stream)), "asgs_uncertainty")


def profile_enable(mask: int):
    check(lib.asgs_profile_enable(mask), "asgs_profile_enable")


def profile_read(kernel_class: int):
    ms, n = C.c_double(), C.c_int64()
    check(lib.asgs_profile_read(kernel_class, C.byref(ms), C.byref(n)), "asgs_profile_read")
    return ms.value, n.value
