"""GPU parity of the render path (projection, binning/sort, blend, backward)
against the FP64 oracle, through the C ABI.

Images: max |x - ref| / max |ref| <= 1e-4 per channel group; gradients
<= 1e-3 per tensor. Pixels with a compositing decision within the guard band
of its threshold (computed by the oracle in FP64) are excluded from image
comparisons and get zero upstream gradient, on both sides; the excluded
fraction is asserted per case. Tile lists and sort order are checked twice:
re-derived from the kernels' own float32 footprint values and depth keys with
integer arithmetic (bit for bit, no exclusion), and against the oracle's
lists, where only Gaussians within the band of a rectangle edge or of a depth
tie (4 float32 ulps) may differ; their number is bounded.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (GRAD_TOL, IMG_TOL, check_binning_self_consistent, check_lists_vs_oracle,
                            guard_report, log, oracle_opts, rel_err, to_np, upstream)

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2505_22335_amd as P
    from paper_2505_22335_amd import _lib as L


def _gpu_render(scene, cams, nf, G=None, **kw):
    g = P.gaussians_to_device(scene.arrays())
    rc = P.RenderContext(cams, scene.n, n_feat=nf, **kw)
    rc.fit(g)
    out = rc.forward(g)
    res = dict(out={k: to_np(v) for k, v in out.items()}, rc=rc, g=g)
    if G is not None:
        V = len(cams)
        dimg = {k: torch.as_tensor(np.stack([G[k]] * V)).cuda() if not isinstance(G[k], list) else
                torch.as_tensor(np.stack(G[k])).cuda() for k in G}
        dg, dpose = rc.backward(g, dimg)
        torch.cuda.synchronize()
        res["dg"] = {k: to_np(v) for k, v in dg.items()}
        res["dpose"] = to_np(dpose)
    torch.cuda.synchronize()
    return res


def _check_lists(rc, ref, label):
    """Self-consistency (exact, no exclusion) and lists vs the oracle (only
    Gaussians at a rectangle edge may differ: plain Gaussians have no depth
    tie band). Returns the cross-precision report."""
    st, _ = check_binning_self_consistent(rc, label)
    rep = check_lists_vs_oracle(rc, ref, st, tie_ulps=0, label=label)
    if rep["rect_band"] == 0:
        assert rep["gpu_isect"] == rep["isect"], rep
    return rep


def _guard(ref, label, max_frac):
    keep, rep = guard_report(ref["margins"], tie_ulps=0)
    log("guard band", label, rep)
    assert rep["frac"] <= max_frac, rep
    return keep


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.2, 0.5, 1.0)])
def test_c1_forward_backward(bg):
    sc, cam, tgt = synth.c1()
    log("case c1", bg)
    nf = 0
    ref = oracle.render_scene(sc, cam, oracle_opts(nf, bg=bg), with_margins=True, keep_lists=True)
    keep = _guard(ref, "c1", 0.01)
    G = upstream(3, cam.height, cam.width, nf)
    for k in G:
        G[k] = G[k] * keep
    res = _gpu_render(sc, [cam], nf, G=G, bg=bg)
    out = res["out"]
    e_rgb = rel_err(out["rgb"][0], ref["rgb"], keep)
    e_d = rel_err(out["depth"][0], ref["depth"], keep)
    e_a = rel_err(out["alpha"][0], ref["alpha"], keep)
    log("c1 image errors rgb %.2e depth %.2e alpha %.2e" % (e_rgb, e_d, e_a))
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_a <= IMG_TOL
    _check_lists(res["rc"], ref, "c1")
    _, gr = oracle.render_scene(sc, cam, oracle_opts(nf, bg=bg), grad_out=G, pose_grad=True)
    for k in ("mean", "scale", "rot", "opacity", "rgb"):
        e = rel_err(res["dg"][k][0], gr["gauss"][k])
        log("c1 grad", k, "%.2e" % e)
        assert e <= GRAD_TOL, k
    e = rel_err(res["dpose"][0], gr["pose"])
    log("c1 pose grad %.2e" % e, res["dpose"][0], gr["pose"])
    assert e <= GRAD_TOL


@pytest.mark.parametrize("case", ["c1", "tiny"])
def test_three_sigma_footprint(case):
    """extent_mode 1 (the vanilla 3-sigma square footprint): images,
    gradients and tile lists against the oracle in the same mode; C1 (10k
    Gaussians, 640x480) and a ragged 16-d feature scene."""
    if case == "c1":
        sc, cam, _ = synth.c1()
        nf = 0
    else:
        nf = 16
        sc = synth.tiny_scene(210, 300, n_feat=nf, logs_mu=-2.6)
        cam = synth.Camera(75, 53, 60.0, 60.0, 37.0, 26.0, np.eye(3, 4, dtype=np.float32))
    log("case three-sigma footprint", case)
    ref = oracle.render_scene(sc, cam, oracle_opts(nf, extent_mode=1), with_margins=True, keep_lists=True)
    keep = _guard(ref, "3sigma " + case, 0.02)
    G = upstream(21, cam.height, cam.width, nf)
    for k in G:
        G[k] = G[k] * keep
    res = _gpu_render(sc, [cam], nf, G=G, extent_mode=1)
    keys = ("rgb", "depth", "alpha") + (("feat",) if nf else ())
    for k in keys:
        e = rel_err(res["out"][k][0], ref[k], keep)
        log("3sigma", case, k, "%.2e" % e)
        assert e <= IMG_TOL, k
    _check_lists(res["rc"], ref, "3sigma " + case)
    _, gr = oracle.render_scene(sc, cam, oracle_opts(nf, extent_mode=1), grad_out=G, pose_grad=True)
    for k in ("mean", "scale", "rot", "opacity", "rgb") + (("feat",) if nf else ()):
        e = rel_err(res["dg"][k][0], gr["gauss"][k])
        log("3sigma grad", case, k, "%.2e" % e)
        assert e <= GRAD_TOL, k
    assert rel_err(res["dpose"][0], gr["pose"]) <= GRAD_TOL


@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_scene_features_ragged(seed):
    """Small image that is not a multiple of the tile size, 16-d features."""
    nf = 16
    sc = synth.tiny_scene(200 + seed, 300, n_feat=nf, logs_mu=-2.6)
    cam = synth.Camera(75, 53, 60.0, 60.0, 37.0, 26.0, np.eye(3, 4, dtype=np.float32))
    log("case tiny", seed)
    ref = oracle.render_scene(sc, cam, oracle_opts(nf), with_margins=True, keep_lists=True)
    keep = _guard(ref, "tiny", 0.02)
    G = upstream(10 + seed, cam.height, cam.width, nf)
    for k in G:
        G[k] = G[k] * keep
    res = _gpu_render(sc, [cam], nf, G=G)
    out = res["out"]
    for k in ("rgb", "depth", "alpha", "feat"):
        e = rel_err(out[k][0], ref[k], keep)
        log("tiny", k, "%.2e" % e)
        assert e <= IMG_TOL, k
    _check_lists(res["rc"], ref, "tiny")
    _, gr = oracle.render_scene(sc, cam, oracle_opts(nf), grad_out=G, pose_grad=True)
    for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
        e = rel_err(res["dg"][k][0], gr["gauss"][k])
        log("tiny grad", k, "%.2e" % e)
        assert e <= GRAD_TOL, k
    assert rel_err(res["dpose"][0], gr["pose"]) <= GRAD_TOL


def test_needle_gaussians_and_faint_opacities():
    """Per-wave culling stress: anisotropic footprints (log-scale spread 1.0
    per axis, axis ratios up to ~200, random rotations) and opacities just
    above alpha_min, whose small ellipses sit near quarter and tile
    boundaries. (With ratios near 1e3 the FP32 rotation gradient through the
    projection loses the 1e-3 budget to conditioning, independent of the
    blend.)"""
    nf = 16
    sc = synth.tiny_scene(321, 400, n_feat=nf, logs_mu=-3.0, logs_sd=1.0)
    rng = np.random.default_rng(5)
    faint = rng.random(sc.opacity.shape) < 0.5
    sc.opacity[faint] = (1.0 / 255.0) * (1.0 + rng.uniform(0.01, 0.3, faint.sum())).astype(np.float32)
    cam = synth.Camera(96, 80, 70.0, 70.0, 47.5, 39.5, np.eye(3, 4, dtype=np.float32))
    log("case needles")
    ref = oracle.render_scene(sc, cam, oracle_opts(nf), with_margins=True, keep_lists=True)
    keep = _guard(ref, "needles", 0.05)
    G = upstream(31, cam.height, cam.width, nf)
    for k in G:
        G[k] = G[k] * keep
    res = _gpu_render(sc, [cam], nf, G=G)
    out = res["out"]
    for k in ("rgb", "depth", "alpha", "feat"):
        e = rel_err(out[k][0], ref[k], keep)
        log("needles", k, "%.2e" % e)
        assert e <= IMG_TOL, k
    _check_lists(res["rc"], ref, "needles")
    _, gr = oracle.render_scene(sc, cam, oracle_opts(nf), grad_out=G, pose_grad=True)
    for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
        e = rel_err(res["dg"][k][0], gr["gauss"][k])
        log("needles grad", k, "%.2e" % e)
        assert e <= GRAD_TOL, k


@pytest.mark.parametrize("n,min_len", [(700, 160), (5000, 2048), (12000, 2048)])
def test_long_tile_lists(n, min_len):
    """Long tile lists from a dense cluster over a 32x32 image (2x2 tiles).
    About 300-450 entries: backward lists walked in three or four segments
    of 128 from the states the forward records at the boundaries. About
    2.5k-3.5k and 6.5k-7.8k entries: longer than one in-LDS sort (two sorted
    runs, one merge; four runs, two merge rounds, a ragged last run), and a
    long last backward segment. Lists bit for bit against their integer
    re-derivation; against the oracle's lists outside the band (with ~7k
    Gaussians per list more of them have a depth neighbour within 4 ulps);
    images and gradients as elsewhere."""
    nf = 16
    sc = synth.tiny_scene(77, n, n_feat=nf, logs_mu=-3.2, logs_sd=0.3, spread=0.25)
    cam = synth.Camera(32, 32, 60.0, 60.0, 15.5, 15.5, np.eye(3, 4, dtype=np.float32))
    log("case long lists", n)
    ref = oracle.render_scene(sc, cam, oracle_opts(nf), with_margins=True, keep_lists=True)
    lens = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    log("list lengths", lens.tolist())
    assert lens.min() > min_len
    keep = _guard(ref, "long lists %d" % n, 0.10)
    G = upstream(41, cam.height, cam.width, nf)
    for k in G:
        G[k] = G[k] * keep
    res = _gpu_render(sc, [cam], nf, G=G)
    _check_lists(res["rc"], ref, "long lists %d" % n)
    for k in ("rgb", "depth", "alpha", "feat"):
        e = rel_err(res["out"][k][0], ref[k], keep)
        log("long lists", k, "%.2e" % e)
        assert e <= IMG_TOL, k
    _, gr = oracle.render_scene(sc, cam, oracle_opts(nf), grad_out=G, pose_grad=True)
    for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
        e = rel_err(res["dg"][k][0], gr["gauss"][k])
        log("long lists grad", k, "%.2e" % e)
        assert e <= GRAD_TOL, k


def test_multiview_batch_equals_single():
    """Three views in one call give the same images and gradients as one call
    per view (results are per view; the batch shares one sort)."""
    nf = 16
    sc = synth.tiny_scene(300, 400, n_feat=nf, logs_mu=-2.6)
    base = np.eye(3, 4, dtype=np.float32)
    cams = [synth.Camera(64, 48, 60.0, 60.0, 31.5, 23.5,
                         synth.perturb_pose(base, [0.05 * v, -0.02 * v, 0.0], [0.0, 0.03 * v, 0.01 * v]))
            for v in range(3)]
    log("case multiview")
    rng = np.random.default_rng(5)
    G = dict(rgb=[rng.normal(size=(3, 48, 64)).astype(np.float32) for _ in cams],
             depth=[rng.normal(size=(48, 64)).astype(np.float32) for _ in cams],
             alpha=[rng.normal(size=(48, 64)).astype(np.float32) for _ in cams],
             feat=[rng.normal(size=(nf, 48, 64)).astype(np.float32) for _ in cams])
    batch = _gpu_render(sc, cams, nf, G=G)
    check_binning_self_consistent(batch["rc"], "multiview batch")
    for v, cam in enumerate(cams):
        Gv = {k: G[k][v] for k in G}
        one = _gpu_render(sc, [cam], nf, G=Gv)
        for k in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(batch["out"][k][v], one["out"][k][0]), (v, k)
        for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
            assert np.array_equal(batch["dg"][k][v], one["dg"][k][0]), (v, k)
        np.testing.assert_allclose(batch["dpose"][v], one["dpose"][0], rtol=1e-6, atol=1e-9)


def test_largest_view_batch_equals_single():
    """The largest batch one call takes (64 views, uploaded to the device in
    chunks of 16): the views at the chunk edges give the same images and
    gradients bitwise as one call per view, the batch's tile lists are
    self-consistent, and one view more is refused."""
    nf = 16
    sc = synth.tiny_scene(64, 300, n_feat=nf, logs_mu=-2.6)
    base = np.eye(3, 4, dtype=np.float32)
    cams = [synth.Camera(32, 24, 30.0, 30.0, 15.5, 11.5,
                         synth.perturb_pose(base, [0.01 * (v % 8), -0.01 * (v // 8), 0.0],
                                            [0.0, 0.004 * (v % 5), 0.003 * (v % 3)]))
            for v in range(L.MAX_VIEWS)]
    log("case largest view batch", len(cams))
    rng = np.random.default_rng(64)
    G = dict(rgb=[rng.normal(size=(3, 24, 32)).astype(np.float32) for _ in cams],
             depth=[rng.normal(size=(24, 32)).astype(np.float32) for _ in cams],
             alpha=[rng.normal(size=(24, 32)).astype(np.float32) for _ in cams],
             feat=[rng.normal(size=(nf, 24, 32)).astype(np.float32) for _ in cams])
    batch = _gpu_render(sc, cams, nf, G=G)
    check_binning_self_consistent(batch["rc"], "largest view batch")
    assert np.any(batch["out"]["alpha"][L.MAX_VIEWS - 1] > 0)
    for v in (0, 15, 16, 17, 47, 48, L.MAX_VIEWS - 1):
        Gv = {k: G[k][v] for k in G}
        one = _gpu_render(sc, [cams[v]], nf, G=Gv)
        for k in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(batch["out"][k][v], one["out"][k][0]), (v, k)
        for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
            assert np.array_equal(batch["dg"][k][v], one["dg"][k][0]), (v, k)
        np.testing.assert_allclose(batch["dpose"][v], one["dpose"][0], rtol=1e-6, atol=1e-9)
    with pytest.raises(L.AsgsError) as ei:
        P.RenderContext(cams + cams[:1], sc.n, n_feat=nf)
    assert ei.value.status == L.E_INVALID


def test_split_lists_batch_invariant_and_deterministic():
    """Lists long enough for the segmented backward (~300-450 entries over a
    32x32 view), three views in one call vs one call per view: images and
    gradients bitwise equal (the split depends only on each view's own
    lists), and a second identical call reproduces the first bitwise."""
    nf = 16
    sc = synth.tiny_scene(77, 700, n_feat=nf, logs_mu=-3.2, logs_sd=0.3, spread=0.25)
    base = np.eye(3, 4, dtype=np.float32)
    cams = [synth.Camera(32, 32, 60.0, 60.0, 15.5, 15.5,
                         synth.perturb_pose(base, [0.004 * v, -0.003 * v, 0.0], [0.0, 0.002 * v, 0.0]))
            for v in range(3)]
    log("case split lists batch invariance")
    rng = np.random.default_rng(9)
    G = dict(rgb=[rng.normal(size=(3, 32, 32)).astype(np.float32) for _ in cams],
             depth=[rng.normal(size=(32, 32)).astype(np.float32) for _ in cams],
             alpha=[rng.normal(size=(32, 32)).astype(np.float32) for _ in cams],
             feat=[rng.normal(size=(nf, 32, 32)).astype(np.float32) for _ in cams])
    batch = _gpu_render(sc, cams, nf, G=G)
    check_binning_self_consistent(batch["rc"], "split lists batch")
    again = _gpu_render(sc, cams, nf, G=G)
    for k in ("rgb", "depth", "alpha", "feat"):
        assert np.array_equal(batch["out"][k], again["out"][k]), k
    for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
        assert np.array_equal(batch["dg"][k], again["dg"][k]), k
    for v, cam in enumerate(cams):
        Gv = {k: G[k][v] for k in G}
        one = _gpu_render(sc, [cam], nf, G=Gv)
        for k in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(batch["out"][k][v], one["out"][k][0]), (v, k)
        for k in ("mean", "scale", "rot", "opacity", "rgb", "feat"):
            assert np.array_equal(batch["dg"][k][v], one["dg"][k][0]), (v, k)


def test_empty_and_offscreen():
    """All Gaussians behind the camera or off screen: zero images, zero grads."""
    sc = synth.tiny_scene(400, 50)
    sc.mean[2] = -sc.mean[2]  # behind the camera
    cam = synth.Camera(40, 30, 40.0, 40.0, 19.5, 14.5, np.eye(3, 4, dtype=np.float32))
    G = upstream(1, 30, 40, 0)
    res = _gpu_render(sc, [cam], 0, G=G)
    assert np.all(res["out"]["rgb"] == 0) and np.all(res["out"]["alpha"] == 0)
    assert all(np.all(v == 0) for v in res["dg"].values())
    assert np.all(res["dpose"] == 0)
    ni, nvis, ov = res["rc"].status()
    assert ni == 0 and nvis == 0
    check_binning_self_consistent(res["rc"], "empty")


def test_capacity_overflow_is_reported():
    sc, cam, _ = synth.c1()
    g = P.gaussians_to_device(sc.arrays())
    rc = P.RenderContext([cam], sc.n, n_feat=0, capacity=1000)
    out = rc.forward(g)
    ni, nvis, ov = rc.status()
    assert ov == 1 and ni > 1000
    need = rc.count(g)
    assert need == ni
