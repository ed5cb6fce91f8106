"""Pins for the oracle's binning and compositing (Sec. 3.1 Eq. 3, Eq. 10).

Brute-force per-pixel compositing without tiles or keys; tile-size
invariance; closed forms for identical stacked footprints; invariants
(alpha = 1 - T_final, constant colour).
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import RenderOpts, bin_and_sort, composite_bruteforce, composite_tile, render_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cam(w=64, h=48, f=60.0):
    return synth.Camera(w, h, f, f, (w - 1) / 2, (h - 1) / 2, np.eye(3, 4, dtype=np.float32))


@pytest.mark.parametrize("seed,nf", [(11, 0), (12, 4), (13, 0)])
def test_tiled_equals_bruteforce(seed, nf):
    sc = synth.tiny_scene(seed, 60, n_feat=nf)
    cam = _cam()
    opts = RenderOpts(n_feat=nf)
    out = render_scene(sc, cam, opts)
    p = out["proj"]
    g = out["gauss"]
    chans = [g["rgb"].T, p["z"].detach().numpy()[:, None]]
    if nf:
        chans.append(g["feat"].T)
    chans = np.concatenate(chans, 1)
    front = p["z"].detach().numpy() > opts.znear
    idx = np.flatnonzero(front)
    acc, asum, Tf = composite_bruteforce(
        p["u"].detach().numpy()[idx], p["v"].detach().numpy()[idx], p["A"].detach().numpy()[idx],
        p["B"].detach().numpy()[idx], p["C"].detach().numpy()[idx], g["opacity"][idx],
        p["z"].detach().numpy()[idx], chans[idx], cam.width, cam.height, opts)
    np.testing.assert_allclose(out["rgb"], acc[..., :3].transpose(2, 0, 1), atol=1e-12)
    np.testing.assert_allclose(out["depth"], acc[..., 3], atol=1e-12)
    np.testing.assert_allclose(out["alpha"], asum, atol=1e-12)
    np.testing.assert_allclose(out["T_final"], Tf, atol=1e-12)
    if nf:
        np.testing.assert_allclose(out["feat"], acc[..., 4:].transpose(2, 0, 1), atol=1e-12)
    assert out["alpha"].max() > 0.5  # the scene actually covers the image


def test_tile_size_invariance():
    sc = synth.tiny_scene(21, 80, n_feat=2)
    cam = _cam(70, 50)
    outs = [render_scene(sc, cam, RenderOpts(tile=t, n_feat=2)) for t in (8, 16, 32)]
    for o in outs[1:]:
        for k in ("rgb", "depth", "feat", "alpha", "T_final"):
            np.testing.assert_allclose(o[k], outs[0][k], atol=1e-12)


def test_alpha_is_one_minus_transmittance():
    sc, cam, _ = synth.c1()
    sub = synth.PlainScene(sc.mean[:, :1500], sc.scale[:, :1500], sc.rot[:, :1500],
                           sc.opacity[:1500], sc.rgb[:, :1500])
    out = render_scene(sub, cam, RenderOpts(n_feat=0))
    np.testing.assert_allclose(out["alpha"], 1.0 - out["T_final"], atol=1e-12)
    assert (out["T_final"] < 1e-3).any()  # some pixels run into termination


def _stack(K, alpha_center, zs, color, W=17, H=17):
    """K Gaussians with one identical footprint centred on a pixel."""
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    u = t(np.full(K, 8.0))
    v = t(np.full(K, 8.0))
    A = t(np.full(K, 0.08))
    B = t(np.full(K, 0.01))
    C = t(np.full(K, 0.05))
    o = t(np.full(K, alpha_center))
    ch = t(np.concatenate([np.tile(color, (K, 1)), np.asarray(zs)[:, None]], 1))
    px, py = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    return u, v, A, B, C, o, ch, t(px.ravel()), t(py.ravel())


@pytest.mark.parametrize("alpha", [0.3, 0.6, 0.95])
def test_identical_stack_closed_form(alpha):
    """K identical footprints (alpha a at a pixel): m = max{j : (1-a)^j >= T_min}
    contribute, C = c (1 - (1-a)^m), D = sum_{j<=m} z_j a (1-a)^(j-1)."""
    K = 40
    zs = np.linspace(1.0, 5.0, K)
    color = np.array([0.2, 0.5, 0.9])
    opts = RenderOpts(n_feat=0)
    args = _stack(K, alpha, zs, color)
    acc, asum, Tf, nc = composite_tile(*args, opts)
    dx = 8.0 - args[7].numpy()
    dy = 8.0 - args[8].numpy()
    a = alpha * np.exp(-0.5 * (0.08 * dx * dx + 0.05 * dy * dy) - 0.01 * dx * dy)
    a = np.minimum(a, 0.99)
    for p in range(a.size):
        ap = a[p]
        if ap < opts.alpha_min:
            assert acc[p].abs().max().item() == 0.0 and nc[p] == 0
            continue
        m = 0
        while m < K and (1 - ap) ** (m + 1) >= opts.T_min:
            m += 1
        assert nc[p] == m
        np.testing.assert_allclose(acc[p, :3].numpy(), color * (1 - (1 - ap) ** m), rtol=1e-12)
        dref = sum(zs[j] * ap * (1 - ap) ** j for j in range(m))
        np.testing.assert_allclose(acc[p, 3].item(), dref, rtol=1e-12)
        np.testing.assert_allclose(asum[p].item(), 1 - (1 - ap) ** m, rtol=1e-12)


def test_constant_colour_scene():
    sc = synth.tiny_scene(31, 70)
    sc.rgb[:] = np.array([[0.25], [0.5], [0.75]], np.float32)
    out = render_scene(sc, _cam(), RenderOpts(n_feat=0))
    np.testing.assert_allclose(out["rgb"], np.array([0.25, 0.5, 0.75])[:, None, None] * out["alpha"],
                               rtol=1e-12, atol=1e-15)


def test_background_adds_transmittance():
    sc = synth.tiny_scene(32, 50)
    cam = _cam()
    o0 = render_scene(sc, cam, RenderOpts(n_feat=0))
    o1 = render_scene(sc, cam, RenderOpts(n_feat=0, bg=(1.0, 0.5, 0.0)))
    np.testing.assert_allclose(o1["rgb"] - o0["rgb"],
                               np.array([1.0, 0.5, 0.0])[:, None, None] * o0["T_final"], atol=1e-12)


def test_binning_against_per_tile_enumeration():
    """lexsort binning equals a plain per-tile scan of every Gaussian."""
    sc = synth.tiny_scene(41, 120)
    cam = _cam(80, 64)
    out = render_scene(sc, cam, RenderOpts(n_feat=0), keep_lists=True)
    p = out["proj"]
    TX, TY = p["tiles_xy"]
    for t in range(TX * TY):
        ty, tx = divmod(t, TX)
        members = [n for n in range(len(p["z32"])) if p["visible"][n]
                   and p["rect"][n][0] <= tx <= p["rect"][n][1] and p["rect"][n][2] <= ty <= p["rect"][n][3]]
        members.sort(key=lambda n: (float(p["z32"][n]), n))
        s, e = out["ranges"][t]
        assert list(out["gids"][s:e]) == members
        assert all(out["tiles"][s:e] == t)


def test_golden_two_gaussians():
    """Hand-derived example (tests/golden/two_gaussians.json): two isotropic
    Gaussians over one pixel, values worked out on paper from Eq. 3."""
    with open(os.path.join(GOLDEN, "two_gaussians.json")) as f:
        gd = json.load(f)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    g = gd["gaussians"]
    args = [t(g[k]) for k in ("u", "v", "A", "B", "C", "o")]
    ch = t(np.concatenate([np.asarray(g["rgb"]), np.asarray(g["z"])[:, None]], 1))
    px, py = t([gd["pixel"][0]]), t([gd["pixel"][1]])
    acc, asum, Tf, nc = composite_tile(*args, ch, px, py, RenderOpts(n_feat=0))
    np.testing.assert_allclose(acc[0, :3].numpy(), gd["expected"]["rgb"], rtol=1e-9)
    np.testing.assert_allclose(acc[0, 3].item(), gd["expected"]["depth"], rtol=1e-9)
    np.testing.assert_allclose(asum[0].item(), gd["expected"]["alpha"], rtol=1e-9)


# ---------------------------------------------------------------------------
# Guard-band margins of composite_tile: hand cases where every decision sits
# at a known relative distance from its threshold. Gaussians are centred on
# the pixel (power = 0), so alpha = min(alpha_max, o) exactly.
# ---------------------------------------------------------------------------
def _centred(ops, zs=None, impact_T=1e-3):
    K = len(ops)
    one = torch.ones(K, dtype=torch.float64)
    u = torch.full((K,), 3.0, dtype=torch.float64)
    v = torch.full((K,), 5.0, dtype=torch.float64)
    o = torch.as_tensor(np.asarray(ops, np.float64))
    z = np.asarray(zs if zs is not None else np.arange(1, K + 1), np.float32)
    chans = torch.stack([one, torch.as_tensor(z.astype(np.float64))], 1)
    px = torch.tensor([3.0], dtype=torch.float64)
    py = torch.tensor([5.0], dtype=torch.float64)
    res = composite_tile(u, v, 0.5 * one, 0.0 * one, 0.5 * one, o, chans, px, py, RenderOpts(n_feat=0),
                         with_margins=True, impact_T=impact_T, z32=z)
    return res[3][0], {k: float(m[0]) for k, m in res[4].items()}


def test_margin_alpha_min():
    am = 1.0 / 255.0
    n, m = _centred([am * 1.01])
    assert n == 1
    assert abs(m["alpha"] - 0.01) < 1e-12
    assert abs(m["clamp"] - abs(am * 1.01 - 0.99) / 0.99) < 1e-12
    # skipped just below the threshold, at the same distance
    n, m = _centred([am * 0.99])
    assert n == 0
    assert abs(m["alpha"] - 0.01) < 1e-12
    assert m["term"] == np.inf  # a skipped Gaussian takes no termination decision


def test_margin_alpha_max():
    n, m = _centred([0.9999])
    assert n == 1
    assert abs(m["clamp"] - 0.0099 / 0.99) < 1e-12


def test_margin_termination_counted_below_impact_T():
    """T after the fourth Gaussian is 1.03e-4 (kept, 3 % above T_min); with
    impact_T = 0.5 only the first Gaussian's alpha decision counts, but the
    termination decisions of all of them do."""
    n, m = _centred([0.9, 0.9, 0.9, 0.897], impact_T=0.5)
    assert n == 4
    T4 = (1 - 0.9) ** 3 * (1 - 0.897)
    assert abs(m["term"] - abs(T4 - 1e-4) / 1e-4) < 1e-9
    assert abs(m["term"] - 0.03) < 1e-9
    assert abs(m["alpha"] - abs(0.9 - 1 / 255) * 255) < 1e-9


def test_margin_of_the_stopping_gaussian():
    """The fourth Gaussian would take T to 5e-5 < T_min: compositing stops
    before it (three contributors) and its decision sits at 0.5."""
    n, m = _centred([0.9, 0.9, 0.9, 0.95])
    assert n == 3
    assert abs(m["term"] - 0.5) < 1e-9


def test_margin_depth_tie_in_ulps():
    z1 = np.float32(1.0)
    z2 = np.float32(z1 + 3 * np.spacing(z1))
    n, m = _centred([0.5, 0.5], zs=[z1, z2])
    assert n == 2 and m["tie"] == 3.0
    # a neighbour that is skipped at the pixel takes no order decision
    n, m = _centred([0.5, 0.001], zs=[z1, z2])
    assert n == 1 and m["tie"] == np.inf
