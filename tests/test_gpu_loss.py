"""GPU: the fused weighted-L1 loss kernel (asgs_l1_loss) against a plain
PyTorch FP32 computation of the same loss and gradient."""
import numpy as np
import pytest
import torch

from tests.gpu_util import log

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2505_22335_amd.core import l1_loss_grad


@pytest.mark.parametrize("V,H,W,use_weight", [(2, 40, 56, True), (3, 23, 37, False)])
def test_l1_loss_matches_torch(V, H, W, use_weight):
    nf = 16
    g = torch.Generator().manual_seed(7)
    mk = lambda *s: torch.rand(*s, generator=g).cuda()
    maps = {"rgb": mk(V, 3, H, W), "depth": mk(V, H, W), "feat": mk(V, nf, H, W), "alpha": mk(V, H, W)}
    tgt = {"rgb": mk(V, 3, H, W), "depth": mk(V, H, W), "feat": mk(V, nf, H, W)}
    tgt["rgb"][:, :, :5] = maps["rgb"][:, :, :5]          # sign(0) = 0 on these pixels
    weight = mk(H, W) if use_weight else None
    scale = {"rgb": 0.5, "depth": 2.0, "feat": 0.25, "alpha": 3.0}
    grad = {k: torch.full_like(v, 7.0) for k, v in maps.items()}
    loss = torch.empty(V, device="cuda")
    log("case l1 loss", V, H, W, use_weight)
    l1_loss_grad(maps, tgt, grad, scale, weight=weight, loss=loss)
    torch.cuda.synchronize()
    ref_loss = torch.zeros(V, device="cuda")
    for k in ("rgb", "depth", "feat"):
        d = maps[k] - tgt[k]
        w = torch.ones(H, W, device="cuda") if weight is None else weight
        w = w if k == "depth" else w[None]
        ref_g = w * torch.sign(d) * np.float32(scale[k])
        assert torch.equal(grad[k], ref_g), k
        ref_loss += (w * d.abs()).reshape(V, -1).sum(1) * scale[k]
    assert torch.equal(grad["alpha"], torch.zeros_like(grad["alpha"]))  # no alpha target: zero gradient
    assert torch.equal(grad["rgb"][:, :, :5], torch.zeros_like(grad["rgb"][:, :, :5]))
    e = ((loss - ref_loss).abs() / ref_loss.abs()).max().item()
    log("l1 loss", loss.tolist(), ref_loss.tolist(), "%.2e" % e)
    assert e <= 1e-5


@pytest.mark.parametrize("nv,use_weight,nf", [(1, True, 16), (3, False, 16), (2, True, 0)])
def test_forward_l1_equals_forward_then_loss(nv, use_weight, nf):
    """asgs_render_forward_l1 gives the images of asgs_render_forward and the
    gradient planes of asgs_l1_loss on them, bitwise; its loss equals the
    loss kernel's up to the order of the FP32 sum. Views of a 40x37 camera
    (ragged tiles), an alpha target on some views' call, no depth target."""
    import synth
    import paper_2505_22335_amd as P
    sc = synth.tiny_scene(11, 500, n_feat=nf, logs_mu=-2.5)
    base = np.eye(3, 4, dtype=np.float32)
    cams = [synth.Camera(40, 37, 40.0, 40.0, 19.5, 18.0,
                         synth.perturb_pose(base, [0.03 * v, 0.0, 0.01 * v], [0.0, 0.02 * v, 0.0]))
            for v in range(nv)]
    H, W = 37, 40
    g = P.gaussians_to_device(sc.arrays())
    rc = P.RenderContext(cams, sc.n, n_feat=nf)
    rc.fit(g)
    gen = torch.Generator().manual_seed(3)
    mk = lambda *s: torch.rand(*s, generator=gen).cuda()
    tgt = {"rgb": mk(nv, 3, H, W), "alpha": mk(nv, H, W)}
    if nf:
        tgt["feat"] = mk(nv, nf, H, W)
    weight = mk(H, W) if use_weight else None
    scale = {"rgb": 0.5, "depth": 2.0, "feat": 0.25, "alpha": 3.0}
    log("case forward_l1", nv, use_weight, nf)
    ref_img = rc.forward(g)
    ref_img = {k: v.clone() for k, v in ref_img.items()}
    ref_grad = {k: torch.full_like(v, 7.0) for k, v in ref_img.items()}
    ref_loss = torch.empty(nv, device="cuda")
    l1_loss_grad(ref_img, tgt, ref_grad, scale, weight=weight, loss=ref_loss)
    grad = {k: torch.full_like(v, 5.0) for k, v in ref_img.items()}
    loss = torch.empty(nv, device="cuda")
    img = rc.forward_l1(g, tgt, grad, scale, weight=weight, loss=loss)
    torch.cuda.synchronize()
    for k in ref_img:
        assert torch.equal(img[k], ref_img[k]), k
        assert torch.equal(grad[k], ref_grad[k]), k
    assert torch.equal(grad["depth"], torch.zeros_like(grad["depth"]))  # no depth target
    e = ((loss - ref_loss).abs() / ref_loss.abs()).max().item()
    log("forward_l1 loss rel err %.2e" % e)
    assert e < 1e-5
