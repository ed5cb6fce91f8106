"""Pins for the oracle's frozen-structure evaluation and its pose gradient at
tracking scale.

With every compositing decision (skip below alpha_min, clamp at alpha_max,
stop below T_min), the tile lists and their order held at the values of a
base evaluation, the rendered maps are smooth in the pose, so central finite
differences match the analytic pose gradient to O(h^2) even where a plain
finite difference crosses thresholds.
"""
import math

import numpy as np
import pytest

import synth
from oracle import RenderOpts, render_scene


def _loss(out, G):
    return sum(float((out[k] * G[k]).sum()) for k in G)


def test_frozen_reproduces_base_and_moves_smoothly():
    sc = synth.tiny_anchor_scene(3, 40, k=4, n_feat=4)
    cam = synth.Camera(48, 40, 50.0, 50.0, 23.5, 19.5, np.eye(3, 4, dtype=np.float32))
    opts = RenderOpts(n_feat=4)
    base = render_scene(sc, cam, opts, keep_structure=True)
    st = base["structure"]
    again = render_scene(sc, cam, opts, structure=st)
    for k in ("rgb", "depth", "feat", "alpha"):
        assert np.array_equal(base[k], again[k]), k
    # away from the base point the frozen images differ from the plain ones
    # only where a decision flips, and both move continuously with the pose
    xi = np.array([1e-3, 0, 0, 0, 0, 0])
    fr = render_scene(sc, cam, opts, xi0=xi, structure=st)
    assert 0 < np.abs(fr["rgb"] - base["rgb"]).max() < 0.1


def test_frozen_fd_matches_pose_gradient_tiny():
    """Tiny scene, large step: plain FD would cross thresholds, frozen FD
    still matches the analytic gradient to second order."""
    sc = synth.tiny_anchor_scene(11, 60, k=5, n_feat=0)
    cam = synth.Camera(64, 48, 60.0, 60.0, 31.5, 23.5,
                       synth.perturb_pose(np.eye(3, 4, dtype=np.float32), [0.03, 0.0, -0.02], [0.0, 0.02, 0.01]))
    opts = RenderOpts(n_feat=0)
    rng = np.random.default_rng(4)
    G = {"rgb": rng.normal(size=(3, 48, 64)), "depth": rng.normal(size=(48, 64)),
         "alpha": rng.normal(size=(48, 64))}
    base = render_scene(sc, cam, opts, keep_structure=True)
    _, gr = render_scene(sc, cam, opts, grad_out=G, pose_grad=True)
    errs = {}
    for h in (1e-3, 5e-4):
        fd = np.zeros(6)
        for j in range(6):
            e = np.zeros(6)
            e[j] = h
            fd[j] = (_loss(render_scene(sc, cam, opts, xi0=e, structure=base["structure"]), G)
                     - _loss(render_scene(sc, cam, opts, xi0=-e, structure=base["structure"]), G)) / (2 * h)
        errs[h] = np.abs(fd - gr["pose"]).max() / np.abs(gr["pose"]).max()
    assert errs[1e-3] < 2e-3, errs
    # the remainder is the O(h^2) term of the central difference: halving h
    # divides it by four
    assert 0.2 * errs[1e-3] < errs[5e-4] < 0.3 * errs[1e-3], errs


@pytest.mark.slow
def test_tracking_pose_gradient_frozen_fd():
    """Tracking-scale pin: the 200k-Gaussian room at 640x480, the start pose
    perturbed by 2 cm / 1 degree, weighted L1 rgb + depth loss against the
    render at the true pose; central FD with h = 1e-4 on each twist
    coordinate, structure frozen, against the analytic gradient."""
    sc, cam_gt, cam0, w, _ = synth.c4()
    opts = RenderOpts(n_feat=0)
    tgt = render_scene(sc, cam_gt, opts)
    img = render_scene(sc, cam0, opts, keep_structure=True)
    P = cam0.width * cam0.height
    G = {"rgb": w[None] * np.sign(img["rgb"] - tgt["rgb"]) / (3 * P),
         "depth": w * np.sign(img["depth"] - tgt["depth"]) / P}
    _, gr = render_scene(sc, cam0, opts, grad_out=G, pose_grad=True)
    h = 1e-4
    fd = np.zeros(6)
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd[j] = (_loss(render_scene(sc, cam0, opts, xi0=e, structure=img["structure"]), G)
                 - _loss(render_scene(sc, cam0, opts, xi0=-e, structure=img["structure"]), G)) / (2 * h)
    rel = np.abs(fd - gr["pose"]).max() / np.abs(gr["pose"]).max()
    print("tracking pose gradient", gr["pose"], "frozen FD", fd, "rel %.2e" % rel)
    assert rel < 2e-4
    assert math.isfinite(rel)
