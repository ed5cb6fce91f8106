"""GPU: the request loop. Results are bitwise the same alone and in the mix
(fused tracking batches, overlapping streams, a capacity re-run); a tracking
request equals the direct decode -> render -> L1 -> backward path; rendered
maps of served requests match the FP64 oracle (FP32 decoder within 1e-4,
BF16 decoder within its stated bound); admission keeps in-flight work within
the arena."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import IMG_TOL, guard_mask, log, oracle_opts, rel_err, to_np

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2505_22335_amd.pipeline import AnchorRenderer, anchors_to_device
    from paper_2505_22335_amd.serve import MAP, TRACK, RequestSpec, Server


def _targets(a, cams):
    """Maps rendered by the FP32 path at the given cameras (request inputs)."""
    r = AnchorRenderer(a, cams)
    r.fit()
    img = r.forward()
    torch.cuda.synchronize()
    return ([img["rgb"][v].clone() for v in range(len(cams))], [img["depth"][v].clone() for v in range(len(cams))],
            [img["feat"][v].clone() for v in range(len(cams))])


def _jitter(cam, seed, rho=0.01, phi=0.006):
    rng = np.random.default_rng(seed)
    u, e = rng.normal(size=3), rng.normal(size=3)
    return cam.copy_with(synth.perturb_pose(cam.T_wc, rho * u / np.linalg.norm(u), phi * e / np.linalg.norm(e)))


class Workload:
    def __init__(self, n_anchors=10_000, seed=12):
        self.sc, _, _ = synth.c2("shell", n_anchors, seed=seed)
        self.a = anchors_to_device(self.sc)
        poses = synth.trajectory(5)[:12]
        self.full = [synth.camera_c2(T) for T in poses]
        self.half = [synth.camera_half(T) for T in poses]
        self.tf = _targets(self.a, self.full)
        self.th = _targets(self.a, self.half)
        self.weight = torch.as_tensor(np.random.default_rng(3).uniform(size=(480, 640)),
                                      dtype=torch.float32).cuda()

    def track(self, i, images=True):
        cam = _jitter(self.full[i], 100 + i)
        kw = {}
        if images:
            kw = dict(out_rgb=[torch.empty(3, 480, 640, device="cuda")],
                      out_depth=[torch.empty(480, 640, device="cuda")])
        return RequestSpec(TRACK, [cam], [self.tf[0][i]], [self.tf[1][i]], target_feat=[self.tf[2][i]],
                           weight=self.weight, d_pose=torch.empty(1, 6, device="cuda"),
                           loss=torch.empty(1, device="cuda"), **kw)

    def map(self, idx, half):
        cams = [_jitter((self.half if half else self.full)[i], 200 + i) for i in idx]
        t = self.th if half else self.tf
        A, n, npar = self.a.A, self.a.A * self.a.k, self.a.params.numel()
        return RequestSpec(MAP, cams, [t[0][i] for i in idx], [t[1][i] for i in idx],
                           target_feat=[t[2][i] for i in idx], d_pose=torch.empty(len(idx), 6, device="cuda"),
                           loss=torch.empty(len(idx), device="cuda"), d_xyz=torch.empty(3, A, device="cuda"),
                           d_feat=torch.empty(A, 32, device="cuda"), d_off=torch.empty(3, n, device="cuda"),
                           d_params=torch.empty(npar, device="cuda"))


def _outputs(spec):
    out = {"d_pose": spec.d_pose, "loss": spec.loss}
    for k in ("d_xyz", "d_feat", "d_off", "d_params"):
        if getattr(spec, k) is not None:
            out[k] = getattr(spec, k)
    if spec.out_rgb:
        out["rgb"], out["depth"] = spec.out_rgb[0], spec.out_depth[0]
    return {k: to_np(v) for k, v in out.items()}


@pytest.fixture(scope="module")
def wl():
    return Workload()


def test_results_same_alone_and_in_the_mix(wl):
    def specs():
        return ([wl.track(i) for i in range(6)] + [wl.map([0, 3, 6, 9], True), wl.map([1, 4, 7, 10, 11], False)]
                + [wl.track(i) for i in range(6, 10)])
    log("case serve invariance")
    alone_specs = specs()
    with Server(wl.a, n_streams=1, max_batch_views=1, fifo=True, arena_bytes=8 << 30) as s:
        for sp in alone_specs:
            r = s.wait(s.submit(sp))
            assert r.status == 0 and r.batch_views == len(sp.cams)
    torch.cuda.synchronize()
    alone = [_outputs(sp) for sp in alone_specs]
    mixed_specs = specs()
    for sp in mixed_specs:
        sp.arrival = 0.0
    with Server(wl.a, n_streams=3, max_batch_views=16, arena_bytes=8 << 30) as s:
        res = s.replay(mixed_specs)
        st = s.stats()
    torch.cuda.synchronize()
    assert all(r.status == 0 for r in res)
    log("mixed: batches", st.batches, "views", st.batch_views, "max in flight", st.max_in_flight,
        "batch sizes", [r.batch_views for r in res])
    assert max(r.batch_views for r, sp in zip(res, mixed_specs) if sp.kind == TRACK) > 1
    for i, sp in enumerate(mixed_specs):
        got = _outputs(sp)
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (i, k, np.abs(got[k] - alone[i][k]).max())
    # the losses are those of the requests' residuals
    assert all(np.all(o["loss"] > 0) for o in alone)


def test_tracking_request_equals_direct_path(wl):
    sp = wl.track(2, images=False)
    with Server(wl.a, n_streams=2, arena_bytes=4 << 30) as s:
        assert s.wait(s.submit(sp)).status == 0
    torch.cuda.synchronize()
    r = AnchorRenderer(wl.a, sp.cams)
    r.fit()
    img = r.forward()
    HW = 480 * 640
    w = wl.weight
    dimg = {"rgb": w * torch.sign(img["rgb"] - wl.tf[0][2][None]) * np.float32(1.0 / (3 * HW)),
            "depth": w * torch.sign(img["depth"] - wl.tf[1][2][None]) * np.float32(1.0 / HW),
            "feat": w * torch.sign(img["feat"] - wl.tf[2][2][None]) * np.float32(1.0 / (16 * HW)),
            "alpha": torch.zeros_like(img["alpha"])}
    g = r.backward(dimg)
    torch.cuda.synchronize()
    e = rel_err(to_np(sp.d_pose[0]), to_np(g["d_pose"][0]))
    log("served vs direct d_pose", to_np(sp.d_pose[0]), to_np(g["d_pose"][0]), "%.2e" % e)
    assert e <= 1e-6


def test_capacity_rerun_gives_the_same_result(wl):
    """A first request that sees nothing sets a tiny intersection estimate;
    the next one overflows its reservation, is detected at completion and run
    again with the exact count."""
    away = wl.full[0].copy_with(synth.look_at((0.0, 0.0, -6.0), (0.0, 0.0, -9.0), (0.0, -1.0, 0.0)))
    empty = RequestSpec(TRACK, [away], [wl.tf[0][0]], [wl.tf[1][0]], d_pose=torch.empty(1, 6, device="cuda"))
    sp = wl.track(4, images=True)
    ref = wl.track(4, images=True)
    with Server(wl.a, n_streams=1, arena_bytes=4 << 30) as s:
        assert s.wait(s.submit(empty)).status == 0
        r = s.wait(s.submit(sp))
        st = s.stats()
    with Server(wl.a, n_streams=1, arena_bytes=4 << 30) as s:
        assert s.wait(s.submit(ref)).status == 0
    torch.cuda.synchronize()
    log("rerun: attempts", r.attempts, "reruns", st.reruns)
    assert r.status == 0 and r.attempts == 2 and st.reruns == 1
    a, b = _outputs(sp), _outputs(ref)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_admission_under_a_tight_arena(wl):
    specs = [wl.track(i, images=False) for i in range(8)]
    for sp in specs:
        sp.arrival = 0.0
    with Server(wl.a, n_streams=4, max_batch_views=4, arena_bytes=900 << 20) as s:
        res = s.replay(specs)
        st = s.stats()
    log("tight arena: peak MiB", st.arena_peak >> 20, "in flight", st.max_in_flight, "batches", st.batches)
    assert all(r.status == 0 for r in res)
    assert st.arena_peak <= st.arena_bytes


@pytest.mark.slow
@pytest.mark.parametrize("precision,tol", [(0, IMG_TOL), (1, 5e-3)])
def test_served_maps_match_oracle(precision, tol):
    """500k-Gaussian serving scene: a served tracking request's rendered maps
    against the FP64 oracle at the same camera (guard-band pixels excluded)."""
    sc, poses = synth.c5()
    a = anchors_to_device(sc)
    cam = _jitter(synth.camera_c2(poses[7]), 7)
    log("case served maps precision", precision)
    tgt = torch.zeros(3, 480, 640, device="cuda")
    tdep = torch.zeros(480, 640, device="cuda")
    sp = RequestSpec(TRACK, [cam], [tgt], [tdep], d_pose=torch.empty(1, 6, device="cuda"),
                     out_rgb=[torch.empty(3, 480, 640, device="cuda")], out_depth=[torch.empty(480, 640, device="cuda")])
    with Server(a, precision=precision, n_streams=2, arena_bytes=8 << 30) as s:
        assert s.wait(s.submit(sp)).status == 0
    torch.cuda.synchronize()
    ref = oracle.render_scene(sc, cam, oracle_opts(0), with_margins=True)
    keep = guard_mask(ref["margins"])
    for k, x in (("rgb", sp.out_rgb[0]), ("depth", sp.out_depth[0])):
        e = rel_err(to_np(x), ref[k], keep)
        log("served %s precision=%d rel err %.3e" % (k, precision, e))
        assert e <= tol, k


@pytest.mark.slow
def test_mapping_request_gradients_match_oracle(wl):
    """One served mapping request (half resolution, the 10k-anchor room):
    its anchor, decoder-parameter and pose gradients against the FP64
    oracle's gradients of the same weighted L1 residual. Pixels in the
    rendering guard band, and pixels where a channel of the oracle's image
    lies within 1e-4 of its target (where the sign of the residual is not
    decided by the rendering alone), get weight 0 in the request and in
    the oracle's upstream gradient."""
    import paper_2505_22335_amd as P
    i = 5
    cam = _jitter(wl.half[i], 300 + i)
    H, W = cam.height, cam.width
    tr, td, tf = (to_np(x[i]) for x in wl.th)
    ref = oracle.render_scene(wl.sc, cam, oracle_opts(16), with_margins=True)
    keep = guard_mask(ref["margins"])
    far = (np.abs(ref["rgb"] - tr).min(0) > 1e-4) & (np.abs(ref["depth"] - td) > 1e-4) & \
        (np.abs(ref["feat"] - tf).min(0) > 1e-4)
    w = np.random.default_rng(4).uniform(size=(H, W)) * keep * far
    log("mapping request: weighted pixels", int((w > 0).sum()), "of", H * W)
    assert (w > 0).mean() > 0.5
    HW = H * W
    G = {"rgb": w * np.sign(ref["rgb"] - tr) / (3 * HW), "depth": w * np.sign(ref["depth"] - td) / HW,
         "feat": w * np.sign(ref["feat"] - tf) / (16 * HW), "alpha": np.zeros((H, W))}
    A, n, npar = wl.a.A, wl.a.A * wl.a.k, wl.a.params.numel()
    sp = RequestSpec(MAP, [cam], [wl.th[0][i]], [wl.th[1][i]], target_feat=[wl.th[2][i]],
                     weight=torch.as_tensor(w, dtype=torch.float32).cuda(), d_pose=torch.empty(1, 6, device="cuda"),
                     loss=torch.empty(1, device="cuda"), d_xyz=torch.empty(3, A, device="cuda"),
                     d_feat=torch.empty(A, 32, device="cuda"), d_off=torch.empty(3, n, device="cuda"),
                     d_params=torch.empty(npar, device="cuda"))
    with Server(wl.a, n_streams=2, arena_bytes=4 << 30) as s:
        assert s.wait(s.submit(sp)).status == 0
    torch.cuda.synchronize()
    _, gr = oracle.render_scene(wl.sc, cam, oracle_opts(16), grad_out=G, pose_grad=True)
    for name in ("xyz", "feat", "off"):
        e = rel_err(to_np(getattr(sp, "d_" + name)), gr["anchor"][name])
        log("mapping request d_%s %.2e" % (name, e))
        assert e <= 1e-3, name
    Wg = P.unpack_params(sp.d_params, wl.sc.k, 16)
    worst = max(rel_err(to_np(Wg[h][k]), gr["weights"][h][k]) for h in Wg for k in Wg[h])
    log("mapping request d_params worst tensor %.2e" % worst)
    assert worst <= 1e-3
    e = rel_err(to_np(sp.d_pose[0]), gr["pose"])
    log("mapping request d_pose %.2e" % e)
    assert e <= 1e-3
