"""Pins of the oracle's feature lift and cosine distillation (Eq. 11, Eq. 12)
against library routines, closed forms and finite differences (CPU only)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn
from scipy.spatial.distance import cosine as scipy_cosine_distance

from oracle.feature import bilinear_weights, cosine_map, distill, lift, relu_margin, upsample


@pytest.mark.parametrize("Hp,Wp,H,W", [(34, 46, 480, 640), (3, 5, 16, 21), (7, 7, 7, 7), (4, 3, 2, 9)])
def test_upsample_matches_torch_interpolate(Hp, Wp, H, W):
    rng = np.random.default_rng(Hp * W)
    g = rng.normal(size=(3, Hp, Wp))
    ours = upsample(g, H, W).numpy()
    ref = Fnn.interpolate(torch.as_tensor(g)[None], size=(H, W), mode="bilinear", align_corners=False)[0].numpy()
    assert np.abs(ours - ref).max() < 1e-12


def test_upsample_closed_forms():
    # constant grid stays constant; same size is the identity; a ramp is reproduced inside
    assert np.allclose(upsample(np.full((1, 3, 4), 2.5), 30, 40).numpy(), 2.5)
    g = np.random.default_rng(0).normal(size=(2, 5, 6))
    assert np.abs(upsample(g, 5, 6).numpy() - g).max() == 0.0
    ramp = np.arange(8, dtype=np.float64)[None, None, :].repeat(2, 1)
    up = upsample(ramp, 2, 32).numpy()[0, 0]
    x = np.arange(32)
    inside = (x >= 2) & (x <= 29)
    assert np.abs(up[inside] - ((x[inside] + 0.5) / 4 - 0.5)).max() < 1e-14
    i0, i1, w1 = bilinear_weights(32, 8)
    assert i0[0] == 0 and w1[0] == 0.0 and i1[-1] == 7


def test_lift_matches_conv1x1_and_zero_weights():
    rng = np.random.default_rng(1)
    Ft = rng.normal(size=(16, 5, 7))
    W1, b1 = rng.normal(size=(128, 16)), rng.normal(size=128)
    W2, b2 = rng.normal(size=(40, 128)), rng.normal(size=40)
    ours = lift(Ft, W1, b1, W2, b2).numpy()
    x = torch.as_tensor(Ft)[None]
    h = Fnn.relu(Fnn.conv2d(x, torch.as_tensor(W1)[:, :, None, None], torch.as_tensor(b1)))
    ref = Fnn.conv2d(h, torch.as_tensor(W2)[:, :, None, None], torch.as_tensor(b2))[0].numpy()
    assert np.abs(ours - ref).max() < 1e-11
    z = lift(Ft, W1, b1, np.zeros_like(W2), b2).numpy()
    assert np.abs(z - b2[:, None, None]).max() == 0.0
    z1 = lift(Ft, np.zeros_like(W1), b1, W2, b2).numpy()
    assert np.abs(z1 - (W2 @ np.maximum(b1, 0) + b2)[:, None, None]).max() < 1e-12


def test_cosine_map_against_scipy():
    rng = np.random.default_rng(2)
    F, G = rng.normal(size=(384, 3, 4)), rng.normal(size=(384, 3, 4))
    c = cosine_map(torch.as_tensor(F), torch.as_tensor(G)).numpy()
    for y in range(3):
        for x in range(4):
            assert abs(c[y, x] - (1 - scipy_cosine_distance(F[:, y, x], G[:, y, x]))) < 1e-13


def _identity_lift(C=16, s=10.0):
    """W1, b1, W2, b2 with F^ = F~ exactly for inputs above -s: the first C
    hidden units carry F~ + s, the second layer removes s."""
    W1 = np.zeros((128, C))
    W1[:C, :C] = np.eye(C)
    b1 = np.zeros(128)
    b1[:C] = s
    W2 = np.zeros((C, 128))
    W2[:, :C] = np.eye(C)
    return W1, b1, W2, -s * np.ones(C)


def test_distill_closed_forms():
    """F^ = F (grid at full resolution equal to F~): cos = 1, loss 0; with
    the second layer negated, cos = -1 and loss 2."""
    rng = np.random.default_rng(3)
    Ft = rng.normal(size=(16, 6, 8))
    W1, b1, W2, b2 = _identity_lift()
    r = distill(Ft, W1, b1, W2, b2, Ft)
    assert np.abs(r["cos"] - 1).max() < 1e-12 and abs(r["loss"]) < 1e-12
    r2 = distill(Ft, W1, b1, -W2, -b2, Ft)
    assert np.abs(r2["cos"] + 1).max() < 1e-12 and abs(r2["loss"] - 2) < 1e-12


def test_distill_gradients_by_finite_differences():
    rng = np.random.default_rng(4)
    H, W, Nh = 4, 5, 24
    Ft = rng.normal(size=(16, H, W))
    W1, b1 = rng.normal(size=(128, 16)) * 0.3, rng.normal(size=128) * 0.3
    W2, b2 = rng.normal(size=(Nh, 128)) * 0.1, rng.normal(size=Nh) * 0.1
    grid = rng.normal(size=(Nh, 3, 2))
    G = rng.normal(size=(H, W))
    r = distill(Ft, W1, b1, W2, b2, grid, d_cos=G)
    args = dict(feat=Ft, W1=W1, b1=b1, W2=W2, b2=b2)
    h = 1e-6
    for name, a in args.items():
        flat = a.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            def f(delta):
                b = {k: v.copy() for k, v in args.items()}
                b[name].reshape(-1)[idx] += delta
                c = distill(b["feat"], b["W1"], b["b1"], b["W2"], b["b2"], grid)["cos"]
                return float((c * G).sum())
            fd = (f(h) - f(-h)) / (2 * h)
            an = r["grads"][name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)


def test_relu_margin_closed_form():
    """One pixel: unit 0 has z = 0.5 - 0.25 against terms of size 0.75
    (margin 1/3), unit 1 first z = 1e-6 against 1e-6 (margin 1), then
    z = 1 - (1 - 1e-6) against 2 - 1e-6; the other units z = 1 = their scale."""
    Ft = np.zeros((16, 1, 1))
    Ft[0] = 1.0
    W1 = np.zeros((128, 16))
    b1 = np.full(128, 1.0)  # other units: margin 1
    W1[0, 0], b1[0] = 0.5, -0.25
    W1[1, 0], b1[1] = 1e-6, 0.0
    W1[1, 1] = 5.0  # multiplies a zero input: no contribution to z or to the scale
    m = relu_margin(Ft, W1, b1)
    assert abs(m[0, 0] - 1.0 / 3.0) < 1e-12
    W1[1, 0], b1[1] = 1.0, -1.0 + 1e-6  # z = 1e-6, scale = 2 - 1e-6
    m = relu_margin(Ft, W1, b1)
    assert abs(m[0, 0] / (1e-6 / (2 - 1e-6)) - 1) < 1e-9  # z carries the rounding of 1 - 1e-6
