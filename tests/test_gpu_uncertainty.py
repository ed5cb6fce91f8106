"""GPU: the uncertainty MLP F_u, its loss L_u and the motion mask
(asgs_uncertainty; Sec. 3.2 Eq. 5, Sec. 3.3 Eq. 13) against the FP64
oracle, through the C ABI.

sigma within 1e-5 relative per view; the mask bit for bit outside the band
|2 sigma^2 - 1| <= 1e-5 of the oracle; L_u within 1e-5 relative; each
parameter-gradient element within 1e-5 of the tensor's largest magnitude
plus the oracle's bound on what hidden units whose ReLU decision lies within
single-precision reach of zero (2e-5 of the pre-activation's term sizes,
which covers the FP32 upsampling coordinates) can contribute either way.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import log, rel_err, to_np

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2505_22335_amd import _lib as L
    from paper_2505_22335_amd.core import UncertaintyMLP

SIG_TOL = 1e-5
GRAD_TOL = 1e-5


def _pack(m):
    return np.concatenate([m["W1"].ravel(), m["b1"], m["w2"], m["b2"]]).astype(np.float32)


@pytest.mark.parametrize("V,H,W,gh,gw,nh", [(1, 37, 53, 3, 4, 48), (2, 64, 80, 5, 6, 384), (1, 16, 16, 1, 1, 16),
                                            (1, 40, 130, 3, 9, 32), (1, 480, 640, 34, 46, 384),
                                            (64, 16, 16, 1, 1, 16)])
def test_uncertainty_matches_oracle(V, H, W, gh, gw, nh):
    """Ragged tiles, several views, one patch, a grid near the finest allowed,
    the full frame with the 34 x 46 DINO grid, and 64 views (the most a
    call takes)."""
    log("case uncertainty", V, H, W, gh, gw, nh)
    m = synth.uncertainty_inputs(700 + V * H + W, V, H, W, gh, gw, nh)
    u = UncertaintyMLP(V, W, H, nh, gh, gw)
    dev = lambda a: torch.as_tensor(a).cuda()
    out = u(dev(_pack(m)), dev(m["dino"]), dev(m["R"]))
    torch.cuda.synchronize()
    gsum, bsum = None, None
    for v in range(V):
        ref = oracle.uncertainty_loss(m["dino"][v], m["W1"], m["b1"], m["w2"], float(m["b2"][0]), m["R"][v])
        es = rel_err(to_np(out["sigma"][v]), ref["sigma"])
        band = np.abs(2 * ref["sigma"] ** 2 - 1) <= 1e-5
        mism = int(((out["dynamic"][v].cpu().numpy() != 0) != ref["dynamic"])[~band].sum())
        el = abs(float(out["loss"][v]) - ref["loss"]) / max(abs(ref["loss"]), 1e-12)
        b = oracle.uncertainty_flip_bound(m["dino"][v], m["W1"], m["b1"], m["w2"], float(m["b2"][0]), m["R"][v])
        log("uncertainty view", v, "sigma %.2e loss %.2e (gpu %.7f ref %.7f)" % (es, el, float(out["loss"][v]),
                                                                               ref["loss"]),
            "dynamic", int(ref["dynamic"].sum()), "band", int(band.sum()), "mismatches", mism)
        assert es <= SIG_TOL and el <= SIG_TOL and mism == 0
        assert band.sum() <= 1e-4 * band.size + 2
        g = ref["grads"]
        gsum = g if gsum is None else {k: gsum[k] + g[k] for k in g}
        bsum = b if bsum is None else {k: bsum[k] + b[k] for k in b}
    d = to_np(out["d_params"]).astype(np.float64)
    o = 0
    for key, shape in (("W1", (128, nh)), ("b1", (128,)), ("w2", (128,)), ("b2", (1,))):
        n = int(np.prod(shape))
        x, r = d[o:o + n].reshape(shape), np.reshape(gsum[key], shape)
        bound = np.reshape(bsum[key], shape) if key != "b2" else np.zeros(shape)
        scale = max(np.abs(r).max(), 1e-12)
        excess = (np.abs(x - r) - bound) / scale
        log("uncertainty d_%s %.2e" % (key, rel_err(x, r)), "beyond the ReLU bound %.2e" % excess.max(),
            "(hidden units near zero: %d)" % bsum["pairs"])
        assert excess.max() <= GRAD_TOL, (key, excess.max())
        o += n


def test_uncertainty_outputs_optional_and_grid_check():
    """sigma alone (no R) equals the full call's sigma; a grid finer than a
    16-pixel tile can cover is refused before launch."""
    m = synth.uncertainty_inputs(9, 1, 33, 47, 4, 5, 32)
    u = UncertaintyMLP(1, 47, 33, 32, 4, 5)
    dev = lambda a: torch.as_tensor(a).cuda()
    full = u(dev(_pack(m)), dev(m["dino"]), dev(m["R"]))
    only = u(dev(_pack(m)), dev(m["dino"]))
    torch.cuda.synchronize()
    assert torch.equal(full["sigma"], only["sigma"]) and torch.equal(full["dynamic"], only["dynamic"])
    with pytest.raises(L.AsgsError) as ei:
        UncertaintyMLP(1, 40, 40, 32, 30, 30)(dev(np.zeros(128 * 32 + 257, np.float32)),
                                             dev(np.zeros((1, 32, 30, 30), np.float32)))
    assert ei.value.status == L.E_UNSUPPORTED
