"""Pins for the oracle's projection (Sec. 3.1, Eq. 2) and footprint.

Closed forms: on-axis isotropic and axis-aligned off-axis Gaussians; rotation
matrices against scipy; world-frame invariance; footprint tightness and
completeness by brute force over pixels.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import synth
from oracle import RenderOpts, project, quat_to_rotmat, pose_cw, se3_exp

F64 = torch.float64


def _proj(mean, scale, q, o, T_wc, cam, opts):
    R_cw, t_cw = pose_cw(T_wc)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    return project(t(mean), t(scale), t(q), t(o), R_cw, t_cw, cam.width, cam.height,
                   cam.fx, cam.fy, cam.cx, cam.cy, opts)


def test_quat_matches_scipy():
    rng = np.random.default_rng(7)
    q = rng.normal(size=(50, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = quat_to_rotmat(torch.as_tensor(q)).numpy()
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy is scalar-last
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_se3_exp_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(5):
        xi = rng.normal(size=6) * 0.3
        E = se3_exp(torch.as_tensor(xi)).numpy()
        # closed form via synth.perturb_pose applied to the identity pose
        Twc = synth.perturb_pose(np.eye(3, 4, dtype=np.float32), xi[:3], xi[3:]).astype(np.float64)
        Rcw = Twc[:, :3].T
        tcw = -Rcw @ Twc[:, 3]
        np.testing.assert_allclose(E[:3, :3], Rcw, atol=2e-7)
        np.testing.assert_allclose(E[:3, 3], tcw, atol=2e-7)


def test_isotropic_on_axis_closed_form():
    cam = synth.Camera(64, 48, 60.0, 70.0, 31.5, 23.5, np.eye(3, 4, dtype=np.float32))
    opts = RenderOpts(n_feat=0)
    rng = np.random.default_rng(0)
    z = np.array([1.0, 2.5, 4.0])
    s = np.array([0.05, 0.02, 0.1])
    q = rng.normal(size=(3, 4))
    mean = np.stack([np.zeros(3), np.zeros(3), z], 1)
    scale = np.stack([s, s, s], 1)
    p = _proj(mean, scale, q, np.full(3, 0.7), cam.T_wc, cam, opts)
    sxx = (cam.fx * s / z) ** 2 + 0.3
    syy = (cam.fy * s / z) ** 2 + 0.3
    np.testing.assert_allclose(p["A"].numpy(), 1 / sxx, rtol=1e-12)
    np.testing.assert_allclose(p["C"].numpy(), 1 / syy, rtol=1e-12)
    np.testing.assert_allclose(p["B"].numpy(), 0, atol=1e-12)
    np.testing.assert_allclose(p["u"].numpy(), cam.cx)
    np.testing.assert_allclose(p["v"].numpy(), cam.cy)
    np.testing.assert_allclose(p["z"].numpy(), z)


def test_axis_aligned_off_axis_closed_form():
    cam = synth.Camera(640, 480, 525.0, 500.0, 319.5, 239.5, np.eye(3, 4, dtype=np.float32))
    opts = RenderOpts(n_feat=0)
    rng = np.random.default_rng(1)
    n = 20
    z = rng.uniform(1, 4, n)
    x = rng.uniform(-0.5, 0.5, n) * z
    y = rng.uniform(-0.4, 0.4, n) * z
    s = rng.uniform(0.01, 0.1, (n, 3))
    q = np.tile([1.0, 0, 0, 0], (n, 1))
    p = _proj(np.stack([x, y, z], 1), s, q, np.full(n, 0.5), cam.T_wc, cam, opts)
    fx, fy = cam.fx, cam.fy
    a = (fx / z) ** 2 * (s[:, 0] ** 2 + (x / z) ** 2 * s[:, 2] ** 2) + 0.3
    c = (fy / z) ** 2 * (s[:, 1] ** 2 + (y / z) ** 2 * s[:, 2] ** 2) + 0.3
    b = (fx * fy / z**2) * (x * y / z**2) * s[:, 2] ** 2
    det = a * c - b * b
    np.testing.assert_allclose(p["A"].numpy(), c / det, rtol=1e-10)
    np.testing.assert_allclose(p["B"].numpy(), -b / det, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(p["C"].numpy(), a / det, rtol=1e-10)
    np.testing.assert_allclose(p["u"].numpy(), fx * x / z + cam.cx, rtol=1e-12)
    np.testing.assert_allclose(p["v"].numpy(), fy * y / z + cam.cy, rtol=1e-12)


def test_fov_clamp_only_changes_jacobian():
    """Beyond the clamp the Jacobian uses the clamped x/z; inside it nothing changes."""
    cam = synth.Camera(64, 48, 60.0, 60.0, 31.5, 23.5, np.eye(3, 4, dtype=np.float32))
    lim = 1.3 * 64 / (2 * 60.0)
    z = 2.0
    x_in, x_out = 0.5 * lim * z, 2.0 * lim * z
    s = np.array([[0.05, 0.03, 0.2]] * 2)
    q = np.array([[1.0, 0, 0, 0]] * 2)
    mean = np.array([[x_in, 0.0, z], [x_out, 0.0, z]])
    p1 = _proj(mean, s, q, np.full(2, 0.5), cam.T_wc, cam, RenderOpts(n_feat=0))
    p0 = _proj(mean, s, q, np.full(2, 0.5), cam.T_wc, cam, RenderOpts(n_feat=0, fov_clamp=0.0))
    assert abs(p1["A"][0].item() - p0["A"][0].item()) < 1e-15
    assert abs(p1["A"][1].item() - p0["A"][1].item()) > 1e-6
    xc = lim * z
    a = (60 / z) ** 2 * (s[1, 0] ** 2 + (xc / z) ** 2 * s[1, 2] ** 2) + 0.3
    c = (60 / z) ** 2 * s[1, 1] ** 2 + 0.3
    np.testing.assert_allclose(p1["A"][1].item(), 1 / a, rtol=1e-12)  # b == 0 since y == 0
    np.testing.assert_allclose(p1["C"][1].item(), 1 / c, rtol=1e-12)
    np.testing.assert_allclose(p1["u"][1].item(), 60 * x_out / z + 31.5)  # u is unclamped


def test_world_frame_invariance():
    sc = synth.tiny_scene(5, 40)
    cam = synth.Camera(64, 48, 60.0, 60.0, 31.5, 23.5, np.eye(3, 4, dtype=np.float32))
    opts = RenderOpts(n_feat=0)
    p0 = _proj(sc.mean.T, sc.scale.T, sc.rot.T, sc.opacity, cam.T_wc, cam, opts)
    Rg = Rotation.from_rotvec([0.3, -0.7, 0.2]).as_matrix()
    tg = np.array([0.5, -1.0, 2.0])
    mean2 = sc.mean.T.astype(np.float64) @ Rg.T + tg
    qg = Rotation.from_matrix(Rg).as_quat()[[3, 0, 1, 2]]
    qs = sc.rot.T.astype(np.float64)
    # quaternion product qg * q (w,x,y,z)
    w1, x1, y1, z1 = qg
    w2, x2, y2, z2 = qs.T
    q2 = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                   w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)
    T2 = np.zeros((3, 4))
    T2[:, :3] = Rg
    T2[:, 3] = tg
    p1 = _proj(mean2, sc.scale.T, q2, sc.opacity, T2, cam, opts)
    for k in ("u", "v", "A", "B", "C", "z"):
        np.testing.assert_allclose(p1[k].numpy(), p0[k].numpy(), rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(p1["rect"], p0["rect"])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_footprint_tight_and_complete(seed):
    """Every pixel with alpha >= alpha_min lies in the footprint box, and the
    box half-width is the ellipse's exact x/y extent rounded up."""
    sc = synth.tiny_scene(seed, 30, logs_mu=-2.0)
    cam = synth.Camera(96, 80, 70.0, 70.0, 47.5, 39.5, np.eye(3, 4, dtype=np.float32))
    opts = RenderOpts(n_feat=0)
    p = _proj(sc.mean.T, sc.scale.T, sc.rot.T, sc.opacity, cam.T_wc, cam, opts)
    A, B, C = (p[k].numpy() for k in "ABC")
    u, v = p["u"].numpy(), p["v"].numpy()
    o = sc.opacity.astype(np.float64)
    for n in np.flatnonzero(p["visible"]):
        rx, ry = p["radius"][n]
        R = int(max(rx, ry)) + 4
        xs = np.arange(int(np.floor(u[n])) - R, int(np.floor(u[n])) + R + 1)
        ys = np.arange(int(np.floor(v[n])) - R, int(np.floor(v[n])) + R + 1)
        X, Y = np.meshgrid(xs, ys)
        dx, dy = u[n] - X, v[n] - Y
        al = o[n] * np.exp(-0.5 * (A[n] * dx * dx + C[n] * dy * dy) - B[n] * dx * dy)
        hit = al >= opts.alpha_min
        assert np.all(np.abs(X[hit] - np.floor(u[n])) <= rx)
        assert np.all(np.abs(Y[hit] - np.floor(v[n])) <= ry)
        # exact extent of the ellipse d^T K d = kappa^2 along x: sample its boundary
        k2 = 2 * math.log(o[n] / opts.alpha_min)
        K = np.array([[A[n], B[n]], [B[n], C[n]]])
        L = np.linalg.cholesky(np.linalg.inv(K))
        th = np.linspace(0, 2 * np.pi, 20001)
        pts = math.sqrt(k2) * L @ np.stack([np.cos(th), np.sin(th)])
        ex, ey = np.abs(pts[0]).max(), np.abs(pts[1]).max()
        assert rx - 1 < ex + 1e-6 and ex <= rx + 1e-9
        assert ry - 1 < ey + 1e-6 and ey <= ry + 1e-9


def test_culling_rules():
    cam = synth.Camera(64, 48, 60.0, 60.0, 31.5, 23.5, np.eye(3, 4, dtype=np.float32))
    opts = RenderOpts(n_feat=0)
    mean = np.array([[0, 0, 0.1], [0, 0, 2.0], [0, 0, 2.0], [50.0, 0, 2.0], [0, 0, -1.0]])
    s = np.full((5, 3), 0.05)
    q = np.tile([1.0, 0, 0, 0], (5, 1))
    o = np.array([0.9, 0.9, 1.0 / 255.0, 0.9, 0.9])
    p = _proj(mean, s, q, o, cam.T_wc, cam, opts)
    assert p["visible"].tolist() == [False, True, False, False, False]
    assert p["ntiles"][1] >= 1 and p["ntiles"][0] == 0


def test_three_sigma_footprint_closed_form():
    """On-axis isotropic Gaussians (2D covariance s_x^2 + 0.3 and s_y^2 + 0.3,
    no correlation): the 3-sigma square has half side ceil(3 sqrt(l)) in both
    axes with l = mid + sqrt(max(0.1, ((s_x^2 - s_y^2)/2)^2)) (the larger
    eigenvalue, with the vanilla floor of 0.1 on the squared half gap),
    whatever the opacity; the tight box depends on the opacity instead."""
    cam = synth.Camera(640, 480, 500.0, 520.0, 319.5, 239.5, np.eye(3, 4, dtype=np.float32))
    z = np.array([2.0, 3.0, 1.5])
    s = np.array([0.03, 0.011, 0.05])
    mean = np.stack([np.zeros(3), np.zeros(3), z], 1)
    scale = np.stack([s, s, s], 1)
    q = np.tile([1.0, 0.0, 0.0, 0.0], (3, 1))
    sxx = (cam.fx * s / z) ** 2 + 0.3
    syy = (cam.fy * s / z) ** 2 + 0.3
    for o in (0.2, 0.95):
        p = _proj(mean, scale, q, np.full(3, o), cam.T_wc, cam, RenderOpts(n_feat=0, extent_mode=1))
        lmax = 0.5 * (sxx + syy) + np.sqrt(np.maximum(0.1, (0.5 * (sxx - syy)) ** 2))
        r = np.ceil(3 * np.sqrt(lmax))
        np.testing.assert_array_equal(p["radius"][:, 0], r)
        np.testing.assert_array_equal(p["radius"][:, 1], r)
        pt = _proj(mean, scale, q, np.full(3, o), cam.T_wc, cam, RenderOpts(n_feat=0))
        k = math.sqrt(2 * math.log(o * 255.0))
        np.testing.assert_array_equal(pt["radius"][:, 0], np.ceil(k * np.sqrt(sxx)))


def test_three_sigma_footprint_renders_alike_for_faint_gaussians():
    """With every opacity below alpha_min e^4.5 (~0.353) the alpha >= alpha_min
    ellipse lies inside 3 sigma, so both footprints give the same images
    (per-pixel alpha tests decide; the lists differ only by entries that
    contribute nothing)."""
    from oracle import render_scene
    sc = synth.tiny_scene(11, 60, n_feat=0)
    sc.opacity[:] = np.minimum(sc.opacity, 0.34).astype(np.float32)
    cam = synth.Camera(40, 32, 40.0, 40.0, 19.5, 15.5, np.eye(3, 4, dtype=np.float32))
    a = render_scene(sc, cam, RenderOpts(n_feat=0))
    b = render_scene(sc, cam, RenderOpts(n_feat=0, extent_mode=1))
    for key in ("rgb", "depth", "alpha"):
        assert np.abs(a[key] - b[key]).max() < 1e-12, key
