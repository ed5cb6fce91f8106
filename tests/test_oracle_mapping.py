"""Pins of the oracle's mapping losses (Sec. 3.1 Eq. 4, Sec. 3.2 Eq. 5,
Sec. 3.3 Eq. 13 and Eq. 14) against scipy's Gaussian filter, brute-force
window sums, closed forms and finite differences (CPU only)."""
import math

import numpy as np
import pytest
import torch
from scipy.ndimage import gaussian_filter as scipy_gaussian_filter

from oracle.mapping import (MAPPING_WEIGHTS, SSIM_C1, SSIM_C2, gaussian_filter, gaussian_window, mapping_loss,
                            mean_scale, softplus_inverse, ssim_map, uncertainty_loss, uncertainty_mlp)


@pytest.mark.parametrize("H,W", [(20, 23), (7, 5), (1, 12)])
def test_gaussian_filter_matches_scipy_zero_padding(H, W):
    img = np.random.default_rng(H * W).normal(size=(3, H, W))
    ours = gaussian_filter(img).numpy()
    for c in range(3):
        ref = scipy_gaussian_filter(img[c], sigma=1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)
        assert np.abs(ours[c] - ref).max() < 1e-13


def test_window_taps():
    g = gaussian_window()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    assert abs(g[5] / g[6] - math.exp(1 / 4.5)) < 1e-12 and np.allclose(g, g[::-1], rtol=0, atol=0)


def _ssim_brute(x, y, py, px):
    """SSIM of one pixel and channel by explicit window sums (zero outside)."""
    g = gaussian_window()
    H, W = x.shape
    m = dict(x=0.0, y=0.0, xx=0.0, yy=0.0, xy=0.0)
    for i in range(11):
        for j in range(11):
            yy, xx = py + i - 5, px + j - 5
            if 0 <= yy < H and 0 <= xx < W:
                w = g[i] * g[j]
                a, b = x[yy, xx], y[yy, xx]
                m["x"] += w * a
                m["y"] += w * b
                m["xx"] += w * a * a
                m["yy"] += w * b * b
                m["xy"] += w * a * b
    sxx, syy, sxy = m["xx"] - m["x"] ** 2, m["yy"] - m["y"] ** 2, m["xy"] - m["x"] * m["y"]
    return ((2 * m["x"] * m["y"] + SSIM_C1) * (2 * sxy + SSIM_C2)) / \
        ((m["x"] ** 2 + m["y"] ** 2 + SSIM_C1) * (sxx + syy + SSIM_C2))


def test_ssim_against_brute_force_window_sums():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(0, 1, (2, 1, 14, 17))
    s = ssim_map(x, y).numpy()[0]
    for py, px in ((0, 0), (13, 16), (6, 8), (2, 15), (9, 3)):
        assert abs(s[py, px] - _ssim_brute(x[0], y[0], py, px)) < 1e-13


def test_ssim_closed_forms():
    """Equal images: SSIM 1. Constant images a, b: with m the window weight
    inside the image, mu = a m, sigma_x^2 = a^2 (m - m^2), sigma_xy =
    a b (m - m^2); m = 1 away from the border, m = (sum of the taps from the
    centre on)^2 at a corner."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (3, 12, 13))
    assert np.abs(ssim_map(x, x).numpy() - 1).max() < 1e-14
    a, b = 0.7, 0.2
    s = ssim_map(np.full((1, 30, 31), a), np.full((1, 30, 31), b)).numpy()[0]

    def closed(m):
        return ((2 * a * b * m * m + SSIM_C1) * (2 * a * b * (m - m * m) + SSIM_C2)) / \
            (((a * a + b * b) * m * m + SSIM_C1) * ((a * a + b * b) * (m - m * m) + SSIM_C2))
    # (the variance terms cancel to ~1e-16 against C2 = 9e-4: ~1e-13 relative)
    assert abs(s[15, 15] - (2 * a * b + SSIM_C1) / (a * a + b * b + SSIM_C1)) < 1e-12
    assert abs(s[15, 15] - closed(1.0)) < 1e-12
    g = gaussian_window()
    assert abs(s[0, 0] - closed(g[5:].sum() ** 2)) < 1e-12
    assert abs(s[0, 15] - closed(g[5:].sum())) < 1e-12


def test_mapping_loss_closed_forms():
    rng = np.random.default_rng(3)
    H, W = 9, 11
    obs = rng.uniform(0, 1, (3, H, W))
    od = rng.uniform(1, 3, (H, W))
    cos = np.ones((H, W))
    r = mapping_loss(obs, od, obs, od, cos)
    assert abs(r["loss"]) < 1e-14 and np.abs(r["d_rgb"]).max() < 1e-14
    # depth off by 0.5 everywhere, colour exact, features aligned: lam2 / 4
    r = mapping_loss(obs, od + 0.5, obs, od, cos)
    assert abs(r["loss"] - MAPPING_WEIGHTS["lam2"] * 0.25) < 1e-14
    assert np.abs(r["d_depth"] - 2 * 0.5 * MAPPING_WEIGHTS["lam2"] / (H * W)).max() < 1e-16
    # cos = 0: lam4 more; d_cos = -lam4 / HW
    r = mapping_loss(obs, od, obs, od, np.zeros((H, W)))
    assert abs(r["loss"] - MAPPING_WEIGHTS["lam4"]) < 1e-14
    assert np.abs(r["d_cos"] + MAPPING_WEIGHTS["lam4"] / (H * W)).max() < 1e-18
    # every pixel dynamic: nothing left
    r = mapping_loss(rng.uniform(0, 1, (3, H, W)), od + 1, obs, od, cos * 0.3, dynamic=np.ones((H, W), bool))
    assert r["loss"] == 0.0 and not np.any(r["d_rgb"]) and not np.any(r["d_depth"]) and not np.any(r["d_cos"])


def test_mapping_loss_gradients_by_finite_differences():
    rng = np.random.default_rng(4)
    H, W = 8, 9
    rgb, obs = rng.uniform(0, 1, (2, 3, H, W))
    dep, od = rng.uniform(1, 3, (2, H, W))
    cos = rng.uniform(-1, 1, (H, W))
    dyn = rng.uniform(size=(H, W)) < 0.3
    r = mapping_loss(rgb, dep, obs, od, cos, dyn)
    args = dict(rgb=rgb, depth=dep, cos=cos)
    for name, grad in (("rgb", r["d_rgb"]), ("depth", r["d_depth"]), ("cos", r["d_cos"])):
        flat = args[name].reshape(-1)
        for idx in rng.choice(flat.size, size=8, replace=False):
            def f(delta):
                b = {k: v.copy() for k, v in args.items()}
                b[name].reshape(-1)[idx] += delta
                return mapping_loss(b["rgb"], b["depth"], obs, od, b["cos"], dyn)["loss"]
            fd = (f(1e-6) - f(-1e-6)) / 2e-6
            assert abs(fd - grad.reshape(-1)[idx]) <= 1e-8 + 1e-6 * abs(fd), (name, idx)


def test_mean_scale():
    s = np.array([[0.1, 0.3], [0.2, 0.4], [0.6, 0.8]])
    assert abs(mean_scale(s) - 2.4 / 6) < 1e-15


def _fu(rng, Nh=24):
    return (rng.normal(size=(128, Nh)) * 0.2, rng.normal(size=128) * 0.2, rng.normal(size=128) * 0.1,
            float(rng.normal() * 0.1))


def test_uncertainty_mlp_closed_forms():
    """Zero first layer: sigma = sigma_min + softplus(w2 . relu(b1) + b2) at
    every pixel; a constant grid gives a constant map; per pixel it is the
    conv1x1 stack on the upsampled features."""
    rng = np.random.default_rng(5)
    W1, b1, w2, b2 = _fu(rng)
    grid = rng.normal(size=(24, 3, 4))
    s = uncertainty_mlp(grid, np.zeros_like(W1), b1, w2, b2, 10, 13).numpy()
    y = w2 @ np.maximum(b1, 0) + b2
    assert np.abs(s - (1e-3 + math.log1p(math.exp(y)))).max() < 1e-14
    s = uncertainty_mlp(np.ones((24, 3, 4)) * 0.3, W1, b1, w2, b2, 10, 13).numpy()
    assert s.max() - s.min() < 1e-14
    from oracle.feature import upsample
    F = upsample(grid, 10, 13)[None]
    h = torch.relu(torch.nn.functional.conv2d(F, torch.as_tensor(W1)[:, :, None, None], torch.as_tensor(b1)))
    yy = torch.nn.functional.conv2d(h, torch.as_tensor(w2)[None, :, None, None],
                                    torch.tensor([b2], dtype=torch.float64))
    ref = 1e-3 + torch.nn.functional.softplus(yy)[0, 0].numpy()
    assert np.abs(uncertainty_mlp(grid, W1, b1, w2, b2, 10, 13).numpy() - ref).max() < 1e-13
    assert abs(softplus_inverse(0.37) - math.log(math.expm1(0.37))) < 1e-14


def test_uncertainty_loss_minimum_and_mask():
    """Constant sigma = sigma_min + softplus(b2) (zero weights): L_u is
    minimised where sigma^2 = R / lam3 (uniform R), so dL_u/db2 vanishes
    there; the mask is 2 sigma^2 > 1."""
    H, W = 6, 7
    R = np.full((H, W), 0.3)
    lam3 = MAPPING_WEIGHTS["lam3"]
    s_opt = math.sqrt(0.3 / lam3)
    b2 = softplus_inverse(s_opt - 1e-3)
    z = dict(W1=np.zeros((128, 5)), b1=np.zeros(128), w2=np.zeros(128))
    r = uncertainty_loss(np.zeros((5, 2, 2)), z["W1"], z["b1"], z["w2"], b2, R)
    assert abs(r["grads"]["b2"]) < 1e-13
    assert abs(r["loss"] - (0.3 / (2 * s_opt ** 2) + lam3 * math.log(s_opt))) < 1e-14
    assert np.all(r["dynamic"] == (2 * s_opt ** 2 > 1))
    for s0, dyn in ((0.7072, True), (0.7070, False)):
        r = uncertainty_loss(np.zeros((5, 2, 2)), z["W1"], z["b1"], z["w2"], softplus_inverse(s0 - 1e-3), R,
                             need_grad=False)
        assert np.all(r["dynamic"] == dyn)


def test_uncertainty_loss_gradients_by_finite_differences():
    rng = np.random.default_rng(6)
    H, W, Nh = 5, 6, 24
    W1, b1, w2, b2 = _fu(rng, Nh)
    grid = rng.normal(size=(Nh, 2, 3))
    R = rng.uniform(0, 1, (H, W))
    r = uncertainty_loss(grid, W1, b1, w2, b2, R)
    args = dict(W1=W1, b1=b1, w2=w2, b2=np.array([b2]))
    for name, a in args.items():
        flat = a.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            def f(delta):
                b = {k: v.copy() for k, v in args.items()}
                b[name].reshape(-1)[idx] += delta
                return uncertainty_loss(grid, b["W1"], b["b1"], b["w2"], float(b["b2"][0]), R, need_grad=False)["loss"]
            fd = (f(1e-6) - f(-1e-6)) / 2e-6
            an = np.reshape(r["grads"][name], -1)[idx]
            assert abs(fd - an) <= 1e-8 + 1e-6 * abs(an), (name, idx, fd, an)


def test_uncertainty_flip_bound_hand_case():
    """1 x 1 image, one patch with feature (2, -1): unit 0 has z = 2 - 2 = 0
    (in the band), unit 1 z = 2 (far), the others z = b1 = 1. The bound of
    dW1[0] is |dy w2_0| |F| = |dy| 0.5 (2, 1) and of db1[0] |dy| 0.5, with dy
    from sigma = sigma_min + softplus(w2 . relu(z) + b2); nothing else."""
    from oracle.mapping import uncertainty_flip_bound
    grid = np.array([2.0, -1.0]).reshape(2, 1, 1)
    W1 = np.zeros((128, 2))
    W1[0] = (1.0, 0.0)
    W1[1] = (1.0, 1.0)
    b1 = np.ones(128)
    b1[0] = -2.0
    w2 = np.full(128, 0.01)
    w2[0] = 0.5
    R = np.array([[0.3]])
    b = uncertainty_flip_bound(grid, W1, b1, w2, 0.1, R)
    y = 0.01 * (126 + 2) + 0.1  # unit 0 contributes relu(0) = 0
    sig = 1e-3 + math.log1p(math.exp(y))
    dy = (-0.3 / sig ** 3 + MAPPING_WEIGHTS["lam3"] / sig) / (1 + math.exp(-y))
    assert b["pairs"] == 1
    assert np.allclose(b["W1"][0], abs(dy) * 0.5 * np.array([2.0, 1.0]), rtol=1e-14, atol=0)
    assert abs(b["b1"][0] - abs(dy) * 0.5) < 1e-15 and not np.any(b["W1"][1:]) and not np.any(b["b1"][1:])
    assert not np.any(b["w2"])  # |z| = 0 for the banded pair
