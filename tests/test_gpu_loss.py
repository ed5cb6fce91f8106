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
