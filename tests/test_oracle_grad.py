"""Pins for the oracle's backward: central finite differences in float64.

Directional derivatives along seeded random directions, per input tensor, for
plain Gaussians, anchors, head weights and the SE(3) pose twist; plus the
quaternion-normalisation invariant dL/dq . q = 0. Scenes are chosen so that
no compositing decision is within the finite-difference step of its
threshold (asserted from the oracle's own margins).
"""
import copy

import numpy as np
import pytest

import synth
from oracle import RenderOpts, render_scene


def _cam(w=48, h=40, f=50.0):
    return synth.Camera(w, h, f, f, (w - 1) / 2, (h - 1) / 2, np.eye(3, 4, dtype=np.float32))


def _upstream(seed, cam, nf):
    rng = np.random.default_rng(seed)
    G = dict(rgb=rng.normal(size=(3, cam.height, cam.width)),
             depth=rng.normal(size=(cam.height, cam.width)),
             alpha=rng.normal(size=(cam.height, cam.width)))
    if nf:
        G["feat"] = rng.normal(size=(nf, cam.height, cam.width))
    return G


def _loss(out, G):
    s = (out["rgb"] * G["rgb"]).sum() + (out["depth"] * G["depth"]).sum() + (out["alpha"] * G["alpha"]).sum()
    if "feat" in G and "feat" in out:
        s += (out["feat"] * G["feat"]).sum()
    return s


def _f64(scene):
    s = copy.deepcopy(scene)
    for k, v in vars(s).items():
        if isinstance(v, np.ndarray):
            setattr(s, k, v.astype(np.float64))
    if hasattr(s, "weights"):
        s.weights = {h: {k: v.astype(np.float64) for k, v in w.items()} for h, w in s.weights.items()}
    return s


def _check_margins(scene, cam, opts, h):
    out = render_scene(scene, cam, opts, with_margins=True, impact_T=0.0)
    m = out["margins"]
    worst = min(m["alpha"].min(), m["clamp"].min(), m["term"].min())
    assert worst > 1e2 * h, f"scene has a decision within {worst:g} of its threshold"


PLAIN_KEYS = ["mean", "scale", "rot", "opacity", "rgb", "feat"]


@pytest.mark.parametrize("seed", [101, 102])
def test_plain_gradients_fd(seed):
    nf = 3
    sc = _f64(synth.tiny_scene(seed, 25, n_feat=nf, logs_mu=-2.0))
    cam = _cam()
    opts = RenderOpts(n_feat=nf, bg=(0.3, 0.1, 0.7))
    G = _upstream(seed, cam, nf)
    h = 1e-7
    _check_margins(sc, cam, opts, h)
    out, gr = render_scene(sc, cam, opts, grad_out=G, pose_grad=True)
    rng = np.random.default_rng(seed + 7)
    for key in PLAIN_KEYS:
        base = getattr(sc, key)
        d = rng.normal(size=base.shape)
        sp, sm = copy.deepcopy(sc), copy.deepcopy(sc)
        setattr(sp, key, base + h * d)
        setattr(sm, key, base - h * d)
        fd = (_loss(render_scene(sp, cam, opts), G) - _loss(render_scene(sm, cam, opts), G)) / (2 * h)
        an = float((gr["gauss"][key] * d).sum())
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (key, fd, an)
    # pose: central differences along each twist coordinate
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd = (_loss(render_scene(sc, cam, opts, xi0=e), G) - _loss(render_scene(sc, cam, opts, xi0=-e), G)) / (2 * h)
        assert abs(fd - gr["pose"][j]) <= 2e-6 * max(1.0, abs(gr["pose"][j])), (j, fd, gr["pose"][j])


def test_quaternion_gradient_orthogonal_to_q():
    sc = synth.tiny_scene(103, 30, logs_mu=-2.0)
    cam = _cam()
    opts = RenderOpts(n_feat=0)
    out, gr = render_scene(sc, cam, opts, grad_out=_upstream(1, cam, 0))
    dq = gr["gauss"]["rot"]
    dots = (dq * sc.rot.astype(np.float64)).sum(0)
    assert np.abs(dots).max() < 1e-12 * max(1.0, np.abs(dq).max())
    assert np.abs(dq).max() > 1e-6


def test_anchor_gradients_fd():
    nf = 4
    sc = _f64(synth.tiny_anchor_scene(7, 16, k=3, n_feat=nf))
    T_wc = synth.perturb_pose(np.eye(3, 4, dtype=np.float32), [0.05, -0.03, 0.1], [0.02, 0.01, -0.03])
    cam = synth.Camera(48, 40, 50.0, 50.0, 23.5, 19.5, T_wc.astype(np.float64))
    opts = RenderOpts(n_feat=nf)
    G = _upstream(5, cam, nf)
    h = 1e-7
    _check_margins(sc, cam, opts, h)
    out, gr = render_scene(sc, cam, opts, grad_out=G, pose_grad=True)
    assert out["alpha"].max() > 0.3
    rng = np.random.default_rng(9)

    def fd_along(mutate):
        sp, sm = copy.deepcopy(sc), copy.deepcopy(sc)
        mutate(sp, +h)
        mutate(sm, -h)
        return (_loss(render_scene(sp, cam, opts), G) - _loss(render_scene(sm, cam, opts), G)) / (2 * h)

    for key in ("xyz", "feat", "off"):
        d = rng.normal(size=getattr(sc, key).shape)
        fd = fd_along(lambda s, e: setattr(s, key, getattr(s, key) + e * d))
        an = float((gr["anchor"][key] * d).sum())
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (key, fd, an)
    for head in sc.weights:
        for wk in ("W1", "b1", "W2", "b2"):
            d = rng.normal(size=sc.weights[head][wk].shape)

            def mut(s, e, head=head, wk=wk, d=d):
                s.weights[head][wk] = s.weights[head][wk] + e * d
            fd = fd_along(mut)
            an = float((gr["weights"][head][wk] * d).sum())
            assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (head, wk, fd, an)
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd = (_loss(render_scene(sc, cam, opts, xi0=e), G) - _loss(render_scene(sc, cam, opts, xi0=-e), G)) / (2 * h)
        assert abs(fd - gr["pose"][j]) <= 2e-6 * max(1.0, abs(gr["pose"][j])), (j, fd, gr["pose"][j])
