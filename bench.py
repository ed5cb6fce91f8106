"""Throughput of the anchor-Gaussian hot path on one MI355X.

One step = decode (anchor MLPs) -> render forward (project, bin/sort, blend) ->
L1 loss gradient -> render backward -> decode backward, for one batch
of views of a synthetic scene resident in HBM. Prints one JSON line.

Default workload: 20k anchors x 10 = 200k Gaussians on the shell of a
4 x 3 x 3 m room (2 cm grid), one 640x480 view with 16-d features, FP32.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c2s": dict(mode="shell", anchors=20_000, seed=2,
                desc="20k anchors x10 = 200k Gaussians on the room shell, 640x480, 16-d features"),
    "c2v": dict(mode="volume", anchors=20_000, seed=2,
                desc="20k anchors x10 = 200k Gaussians through the room volume, 640x480, 16-d features"),
    "c3": dict(mode="shell", anchors=100_000, seed=3,
               desc="100k anchors x10 = 1M Gaussians on the room shell, 640x480, 16-d features"),
}


VALU_PEAK_OPS = 39.3e12     # FP32 lane-ops/s without packed math (78.6 TFLOP/s counting an FMA as 2)
MFMA_PEAK = {"f32": 157.3e12, "bf16": 2.5e15}  # dense FLOP/s


def algorithmic_bytes(I, nvis, N, A, P, nf=16, l1=True):
    """Minimum bytes each kernel class must move (per launch), from the
    method's data: per intersection a 2D record (u,v,conic,opacity = 6
    floats) plus channels (rgb, depth, feature), per pixel the outputs or the
    upstream gradients, per Gaussian its parameters. With l1, the forward
    also reads the targets of its ch + 1 outputs and writes their L1
    gradients (the fused residual of the benchmark step)."""
    ch = 4 + nf
    rec = 4 * (6 + ch)
    return {
        "blend_fwd": I * rec + I * 4 + P * 4 * (ch + 1 + 2) + (P * 4 * 2 * (ch + 1) if l1 else 0),
        "blend_bwd": I * rec + P * 4 * (ch + 1 + 2) + nvis * rec,
        "project": N * 4 * (3 + 3 + 4 + 1 + 3 + nf) + nvis * rec,
        "sort": N * 8 + I * 12,
        "project_bwd": nvis * rec + N * 4 * (3 + 3 + 4 + 1) + N * 4 * (3 + 3 + 4 + 1 + 3 + nf),
        "decode": A * 4 * (3 + 32 + 30) + N * 4 * (3 + 3 + 4 + 1 + 3 + nf),
        "decode_bwd": N * 4 * (3 + 3 + 4 + 1 + 3 + nf) + A * 4 * 2 * (3 + 32 + 30),
        # rendered rgb, depth, opacity sum, cosine, observed rgb and depth in; R, sigma, mask out
        "residual": P * (4 * (3 + 1 + 1 + 1 + 3 + 1) + 4 + 4 + 1),
    }


def mapping_bytes(P, cells, nh=384, nl=16):
    """Minimum bytes of the mapping-iteration kernels (per launch): the
    feature lift reads the rendered low-dimensional feature and the DINO
    patch grid and writes the cosine (the backward also reads the upstream
    cosine gradient and writes the feature gradient); the mapping loss reads
    rendered and observed colour and depth, the cosine and the mask and
    writes the colour, depth and cosine gradients; the uncertainty MLP reads
    the grid and R and writes sigma and the mask."""
    grid = cells * nh * 4
    return {
        "feature": P * 4 * (nl + 1) + grid,
        "feature_bwd": P * 4 * (nl + 1 + nl) + grid,
        "mapping": P * (4 * (3 + 3 + 1 + 1 + 1 + 3 + 1 + 1) + 1),
        "uncertainty": P * (4 + 4 + 1) + grid,
    }


def mapping_ops(P, cells, nh=384, nl=16):
    """Operation lower bounds of the mapping-iteration kernels: the feature
    lift's first layer per pixel (nl x 128 FMAs, vector) and its second layer
    as the Gram form hT M h (128 x 128, matrix cores; bf16 with three split
    products), the backward twice that; the SSIM window sums (5 maps x 2
    separable 11-tap passes x 3 channels, FP64 at the FP32 vector rate) and
    the backward filter (3 maps x 22 taps x 3 channels); the uncertainty MLP's
    first layer once per patch (nh x 128) and per pixel the interpolation and
    second layer (128 x 6), twice with the gradient."""
    return {
        "feature": {"valu": P * nl * 128, "mfma": P * 2 * 128 * 128 * 3, "mfma_type": "bf16"},
        "feature_bwd": {"valu": 2 * P * nl * 128, "mfma": 2 * P * 2 * 128 * 128 * 3, "mfma_type": "bf16"},
        "mapping": {"valu": P * (5 * 22 * 3 + 3 * 22 * 3)},
        "uncertainty": {"valu": cells * nh * 128 + 2 * P * 128 * 6},
    }


def algorithmic_ops(A, k, V, N, evals, nf=16, precision=0):
    """Lower bounds on the arithmetic of each kernel class (per launch):
    vector lane-op slots (an FMA is one slot, an exponential four) and
    matrix FLOPs with their type. evals = pixel-Gaussian evaluations the
    forward performs at least (sum over pixels of the list position of the
    last composited Gaussian); each needs the offset (2), the conic power
    (5), the alpha_min test (1) and one exponential (4 slots). The decoder's
    two layers per head are dense contractions: 2 (32 * 35 + k m 32) FLOPs
    per anchor and head; its backward is twice that (input and weight
    gradients). Projection: ~200 lane-ops per (view, Gaussian)."""
    ms = (1, 3, 3, 4, nf) if nf else (1, 3, 3, 4)
    dec = A * V * sum(2 * (32 * 35 + k * m * 32) for m in ms)
    dt = "f32" if precision == 0 else "bf16"
    return {
        "blend_fwd": {"valu": 12 * evals},
        "blend_bwd": {"valu": 12 * evals},
        "project": {"valu": 200 * N},
        "project_bwd": {"valu": 400 * N},
        "decode": {"mfma": dec, "mfma_type": dt},
        "decode_bwd": {"mfma": 2 * dec, "mfma_type": "f32"},
    }


def roofline_entry(avg_ms, nbytes, ops):
    """Per-kernel fractions: of HBM (algorithmic bytes / time / 8 TB/s) and of
    the binding roofline (the largest of the HBM, vector-ALU and matrix-core
    lower-bound times, over the measured time)."""
    t = avg_ms * 1e-3
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_valu = ops.get("valu", 0) / VALU_PEAK_OPS
    t_mfma = ops.get("mfma", 0) / MFMA_PEAK[ops.get("mfma_type", "f32")]
    bound = max((t_hbm, "hbm"), (t_valu, "valu"), (t_mfma, "mfma"))
    return {"avg_us": round(avg_ms * 1e3, 2), "alg_bytes": int(nbytes), "valu_ops": int(ops.get("valu", 0)),
            "mfma_flops": int(ops.get("mfma", 0)), "pct_hbm": round(100 * t_hbm / t, 1) if t > 0 else None,
            "bound": bound[1], "pct_bound": round(100 * bound[0] / t, 1) if t > 0 else None}


def measured_traffic(path=os.path.join(ROOT, "profiles", "blend_bwd_c2s_traffic.md")):
    """HBM bytes per blend-backward launch from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when it is missing or the kernel source has
    changed since the counters were taken."""
    import hashlib
    import re
    try:
        txt = open(path).read()
        sha = re.search(r"source_sha256: ([0-9a-f]{64})", txt).group(1)
        src = re.search(r"source: (\S+)", txt).group(1)
        val = float(re.search(r"traffic_bytes_per_launch: ([0-9.]+)", txt).group(1))
        cur = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    except (OSError, AttributeError, ValueError):
        return None
    return val if cur == sha else None


def cpu_baseline(sc, cam, G):
    """The FP64 oracle's forward + backward of the workload's frame on the
    host: median of 3 full frames on all the threads torch uses, and median
    of 3 runs of the frame's central 320x240 quarter (the same rays, a camera
    with the principal point shifted) on one thread."""
    import statistics

    import torch

    import oracle
    import synth
    from oracle import RenderOpts
    threads = torch.get_num_threads()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass

    def timed(c, g):
        t0 = time.perf_counter()
        oracle.render_scene(sc, c, RenderOpts(n_feat=16), grad_out=g, pose_grad=True)
        return time.perf_counter() - t0
    full = [timed(cam, G) for _ in range(3)]
    x0, y0, w, h = cam.width // 4, cam.height // 4, cam.width // 2, cam.height // 2
    quarter = synth.Camera(w, h, cam.fx, cam.fy, cam.cx - x0, cam.cy - y0, cam.T_wc)
    Gq = {k: v[..., y0:y0 + h, x0:x0 + w] for k, v in G.items()}
    torch.set_num_threads(1)
    try:
        one = [timed(quarter, Gq) for _ in range(3)]
    finally:
        torch.set_num_threads(threads)
    mpix, mq = cam.width * cam.height / 1e6, w * h / 1e6
    tf, tq = statistics.median(full), statistics.median(one)
    return {"value": mpix / tf, "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"full {cam.width}x{cam.height} frame, forward+backward incl. decoder and pose gradient, "
                      f"median of 3 on {threads} torch threads",
            "cpu_model": model, "runs_s": [round(x, 2) for x in full],
            "one_core": {"value": mq / tq, "unit": "Mpix/s", "cores": 1,
                         "sample": f"central {w}x{h} quarter of the frame, median of 3 on one thread",
                         "runs_s": [round(x, 2) for x in one]}}


def serving_c5(warmup_s=2.0, measure_s=20.0, burst_s=1.0, seed=5, log=None):
    """The serving mix on the 500k-Gaussian room: Poisson tracking requests
    (one 640x480 view, weighted L1 on rgb/depth/features, pose gradient) at
    300/s and mapping requests (4..16 keyframes at 640x480 or 320x240, anchor
    and MLP gradients) at 20/s, replayed against three server configurations:
    batched with the BF16 decoder, batched with the FP32 decoder, and FP32 one
    request at a time on one stream. Also the saturation throughput of each
    (a burst of burst_s seconds of requests all arriving at once)."""
    import numpy as np
    import torch

    import synth
    from paper_2505_22335_amd.pipeline import AnchorRenderer, anchors_to_device
    from paper_2505_22335_amd.serve import MAP, TRACK, RequestSpec, Server, latency_summary, poisson_arrivals

    sc, poses = synth.c5()
    a = anchors_to_device(sc)
    full = [synth.camera_c2(T) for T in poses]
    half = [synth.camera_half(T) for T in poses]

    def prerender(cams):
        out = ([], [], [])
        for i in range(0, len(cams), 16):
            r = AnchorRenderer(a, cams[i:i + 16])
            r.fit()
            img = r.forward()
            for v in range(img["rgb"].shape[0]):
                out[0].append(img["rgb"][v].clone())
                out[1].append(img["depth"][v].clone())
                out[2].append(img["feat"][v].clone())
            del r, img
        torch.cuda.synchronize()
        return out
    tf, th = prerender(full), prerender(half)
    rng = np.random.default_rng(seed)
    weight = torch.as_tensor(rng.uniform(size=(480, 640)), dtype=torch.float32).cuda()

    def jitter(cam, r):
        u, e = r.normal(size=3), r.normal(size=3)
        return cam.copy_with(synth.perturb_pose(cam.T_wc, 0.01 * u / np.linalg.norm(u),
                                                0.0087 * e / np.linalg.norm(e)))

    T_end = warmup_s + measure_s
    t_tr = poisson_arrivals(rng, 300.0, T_end)
    t_mp = poisson_arrivals(rng, 20.0, T_end)
    events = sorted([(t, TRACK) for t in t_tr] + [(t, MAP) for t in t_mp])
    A, n, npar = a.A, a.A * a.k, a.params.numel()
    d_pose_tr = torch.empty((len(t_tr), 6), device="cuda")
    loss_tr = torch.empty(len(t_tr), device="cuda")
    ring = [dict(d_pose=torch.empty((16, 6), device="cuda"), loss=torch.empty(16, device="cuda"),
                 d_xyz=torch.empty((3, A), device="cuda"), d_feat=torch.empty((A, 32), device="cuda"),
                 d_off=torch.empty((3, n), device="cuda"), d_params=torch.empty(npar, device="cuda"))
            for _ in range(8)]
    specs, kinds, mpix = [], [], []
    it = im = 0
    for t, kind in events:
        r = np.random.default_rng([seed, len(specs)])
        if kind == TRACK:
            i = int(t * 30.0) % 64
            specs.append(RequestSpec(TRACK, [jitter(full[i], r)], [tf[0][i]], [tf[1][i]], target_feat=[tf[2][i]],
                                     weight=weight, d_pose=d_pose_tr[it:it + 1], loss=loss_tr[it:it + 1],
                                     arrival=float(t)))
            it += 1
            mpix.append(0.3072)
        else:
            B = int(r.integers(4, 17))
            small = r.random() < 0.5
            idx = r.choice(64, B, replace=False)
            cams, tg = (half, th) if small else (full, tf)
            o = ring[im % len(ring)]
            specs.append(RequestSpec(MAP, [jitter(cams[j], r) for j in idx], [tg[0][j] for j in idx],
                                     [tg[1][j] for j in idx], target_feat=[tg[2][j] for j in idx],
                                     d_pose=o["d_pose"][:B], loss=o["loss"][:B], d_xyz=o["d_xyz"],
                                     d_feat=o["d_feat"], d_off=o["d_off"], d_params=o["d_params"], arrival=float(t)))
            im += 1
            mpix.append(B * (0.0768 if small else 0.3072))
        kinds.append(kind)
    kinds, mpix = np.array(kinds), np.array(mpix)
    arr = np.array([s.arrival for s in specs])
    offered = float(mpix[arr >= warmup_s].sum() / measure_s)
    modes = {"served_bf16": dict(precision=1, n_streams=3, max_batch_views=16),
             "served_fp32": dict(precision=0, n_streams=3, max_batch_views=16),
             "fifo_fp32": dict(precision=0, n_streams=1, max_batch_views=1, fifo=True)}
    out = {"workload": "50k anchors x10 = 500k Gaussians; Poisson tracking 300/s (640x480, pose grad) + "
                       "mapping 20/s (4-16 keyframes, 640x480 or 320x240, anchor/MLP grads)",
           "warmup_s": warmup_s, "measure_s": measure_s, "requests": len(specs),
           "offered_mpix_s": round(offered, 1), "modes": {}}
    burst = [i for i in range(len(specs)) if arr[i] < burst_s]
    for name, kw in modes.items():
        with Server(a, arena_bytes=32 << 30, **kw) as srv:
            res = srv.replay(specs)
            st = srv.stats()
        done = np.array([r.done for r in res]) - res[0].arrival + arr[0]
        ok = np.array([r.status == 0 for r in res])
        win = arr >= warmup_s
        span = done[win].max() - warmup_s
        summ = latency_summary(res, kinds, t_from=warmup_s)
        # saturation: the first burst_s seconds of requests, all at once
        bspecs = [specs[i] for i in burst]
        saved = [s.arrival for s in bspecs]
        for s_ in bspecs:
            s_.arrival = 0.0
        with Server(a, arena_bytes=32 << 30, **kw) as srv:
            t0 = Server.clock()
            bres = srv.replay(bspecs)
        for s_, t in zip(bspecs, saved):
            s_.arrival = t
        makespan = max(r.done for r in bres) - t0
        out["modes"][name] = {
            "throughput_mpix_s": round(float(mpix[win & ok].sum() / span), 1),
            "saturation_mpix_s": round(float(mpix[burst].sum() / makespan), 1),
            "latency": summ, "batches": int(st.batches), "mean_batch_views": round(st.batch_views / max(st.batches, 1), 2),
            "max_in_flight": int(st.max_in_flight), "arena_peak_gib": round(st.arena_peak / 2 ** 30, 2),
            "reruns": int(st.reruns), "failed": int(st.failed)}
        if log:
            log(name, json.dumps(out["modes"][name]))
    return out


def time_mapping_kernels(r, V, H, W, seed, reps=10):
    """The mapping iteration's kernels on the step's rendered maps (not part
    of the timed step): feature lift forward and backward (N_h 384 on the
    34 x 46 DINO grid of a 476 x 644 crop), the mapping loss with SSIM and
    its gradients, and the uncertainty MLP with L_u's gradient; per class the
    mean launch time from the library's per-launch events."""
    import numpy as np
    import torch

    import synth
    from paper_2505_22335_amd import _lib as L
    from paper_2505_22335_amd.core import FeatureLift, UncertaintyMLP, mapping_loss

    gh, gw, nh = 34, 46, 384
    dev = lambda a: torch.as_tensor(a).cuda()
    fi = synth.feature_inputs(seed + 300, V, H, W, gh, gw, nh)
    fparams = dev(np.concatenate([fi["W1"].ravel(), fi["b1"], fi["W2"].ravel(), fi["b2"]]))
    fl = FeatureLift(V, W, H, nh, gh, gw)
    feat = r.images["feat"].contiguous()
    dino = dev(fi["dino"])
    mm = synth.mapping_maps(seed + 301, V, H, W)
    ui = synth.uncertainty_inputs(seed + 302, V, H, W, gh, gw, nh)
    uparams = dev(np.concatenate([ui["W1"].ravel(), ui["b1"], ui["w2"], ui["b2"]]))
    um = UncertaintyMLP(V, W, H, nh, gh, gw)
    R = dev(ui["R"])
    obs_rgb, obs_depth, dyn = dev(mm["obs_rgb"]), dev(mm["obs_depth"]), dev(mm["dynamic"])
    out = fl.forward(feat, fparams, dino)
    cos = out["cosine"] if isinstance(out, dict) else out[0]
    classes = (L.K_FEATURE, L.K_FEATURE_BWD, L.K_MAPPING, L.K_UNCERTAINTY)
    mask = 0
    for c in classes:
        mask |= 1 << c
    L.profile_enable(mask)
    torch.cuda._sleep(20_000_000)
    for _ in range(reps):
        fl.forward(feat, fparams, dino)
        ml = mapping_loss({"rgb": r.images["rgb"], "depth": r.images["depth"]}, obs_rgb, obs_depth, cosine=cos,
                          dynamic=dyn)
        fl.backward(feat, fparams, dino, ml["d_cos"])
        um(uparams, dino, R)
    torch.cuda.synchronize()
    P, cells = V * H * W, V * gh * gw
    ab, ops = mapping_bytes(P, cells, nh), mapping_ops(P, cells, nh)
    br = {}
    for c, nm in zip(classes, ("feature", "feature_bwd", "mapping", "uncertainty")):
        t, n = L.profile_read(c)
        if n:
            br[nm] = roofline_entry(t / n, ab[nm], ops[nm])
            br[nm]["note"] = "mapping iteration on the step's maps (not part of the timed step)"
    L.profile_enable(0)
    return br


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2s", choices=sorted(WORKLOADS))
    ap.add_argument("--views", type=int, default=1)
    ap.add_argument("--precision", type=int, default=0, help="decoder precision: 0 FP32, 1 BF16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing (counter calibration)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="measured seconds of the serving mix (after 2 s warm-up; 0 = skip)")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving mix (2 s warm-up)")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step into a HIP graph and time its replays (checked bitwise against the eager step)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path is not sharded across GPUs. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2505_22335_amd import _lib as L
    from paper_2505_22335_amd.pipeline import AnchorRenderer, anchors_to_device

    if args.serve_only:
        res = serving_c5(warmup_s=2.0, measure_s=args.serve_seconds or 20.0,
                         log=lambda *m: print(*m, file=sys.stderr, flush=True))
        print(json.dumps({"metric": "p50/p99 request latency, serving mix", "serving": res}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    sc, cam, _ = synth.c2(wl["mode"], wl["anchors"], seed=wl["seed"])
    cams = [cam] if args.views == 1 else [
        cam.copy_with(synth.perturb_pose(cam.T_wc, [0.02 * v, 0.0, 0.01 * v], [0.0, 0.004 * v, 0.0]))
        for v in range(args.views)]
    V, H, W = len(cams), cam.height, cam.width
    rng = np.random.default_rng(wl["seed"] + 100)
    tgt = {"rgb": torch.as_tensor(rng.uniform(size=(V, 3, H, W)), dtype=torch.float32).cuda(),
           "depth": torch.as_tensor(rng.uniform(size=(V, H, W)), dtype=torch.float32).cuda(),
           "feat": torch.as_tensor(rng.uniform(size=(V, 16, H, W)), dtype=torch.float32).cuda(),
           "alpha": torch.as_tensor(rng.uniform(size=(V, H, W)), dtype=torch.float32).cuda()}
    r = AnchorRenderer(anchors_to_device(sc), cams, precision=args.precision)
    r.fit()
    dimg = {k: torch.empty_like(v) for k, v in tgt.items()}
    scale = {k: 1.0 / v.numel() for k, v in tgt.items()}

    def step():
        # render with the L1 residual gradient (mean over each output) formed
        # in the forward's output stage, then the backward
        r.forward_l1(tgt, dimg, scale)
        r.backward(dimg)

    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    I, nvis, ov = r.rc.status()
    if ov:
        raise RuntimeError("intersection capacity exceeded")
    run = step
    if args.graph:
        # The whole step (every library kernel and the loss ops) captured once
        # into a HIP graph and replayed: same work, no per-launch host cost.
        # A replay must reproduce the eager step bitwise.
        ref = {k: v.clone() for k, v in r.images.items()}
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        graph.replay()
        torch.cuda.synchronize()
        for k in ref:
            if not torch.equal(ref[k], r.images[k]):
                raise RuntimeError(f"graph replay differs from the eager step ({k})")
        run = graph.replay
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    # the dominant kernel's mean launch time: HIP events recorded on its launch
    # stream around every blend-backward launch of the same number of steps,
    # launched from the host (a graph replay carries no per-launch events)
    L.profile_enable(1 << L.K_BLEND_BWD)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    bb_ms, bb_n = L.profile_read(L.K_BLEND_BWD)
    L.profile_enable(0)
    N, A, P = r.a.A * r.a.k, r.a.A, V * H * W
    ab = algorithmic_bytes(I, nvis, N * V, A, P)
    dom_ms = bb_ms / max(bb_n, 1)
    achieved = ab["blend_bwd"] / (dom_ms * 1e-3) / 1e9
    mpix = P / 1e6
    res = {
        "metric": "fwd+bwd Mpix/s @640x480, 200k Gaussians",
        "value": round(mpix / (ms * 1e-3), 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 0 else "bf16-decode/f32",
        "precision": ("FP32 arithmetic throughout, except the blend backward's per-entry sums over pixels: "
                      "bf16 matrix cores with both operands split into high and low bfloat16 parts "
                      "(three products, relative error per product below 2^-15)"
                      + ("" if args.precision == 0 else "; decoder forward on bf16 matrix cores")),
        "data": "synthetic",
        "config": {"workload": wl["desc"] + f", {V} view(s), decoder {'FP32' if args.precision == 0 else 'BF16'}",
                   "anchors": A, "gaussians": N, "views": V, "width": W, "height": H, "n_feat": 16,
                   "intersections": I, "visible": nvis},
        "roofline": {"bound": "hbm", "kernel": "blend backward (k_blend_bwd)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if args.workload == "c2s" and V == 1 else None,
                     "avg_ms": round(dom_ms, 5), "launches": bb_n,
                     "algorithmic_bytes": int(ab["blend_bwd"])},
        "wall_s": round(wall, 3),
        "launch": "hip-graph" if args.graph else "host",
    }
    # every kernel class: mean launch time over extra steps with the
    # library's per-launch events, algorithmic bytes and operation lower
    # bounds, fraction of HBM and of the binding roofline
    evals = int(r.rc.array(L.CTX_NCONTRIB, torch.int32).sum().item())
    ops = algorithmic_ops(A, r.a.k, V, N * V, evals, precision=args.precision)
    rm = synth.residual_maps(wl["seed"] + 200, V, H, W)
    obs = {k: torch.as_tensor(rm[k]).cuda() for k in ("cosine", "obs_rgb", "obs_depth")}
    res_out = dict(R=torch.empty((V, H, W), device="cuda"), sigma=torch.empty((V, H, W), device="cuda"),
                   dynamic=torch.empty((V, H, W), dtype=torch.uint8, device="cuda"),
                   xi=torch.empty(V, device="cuda"),
                   work=torch.empty(L.residual_work_size(V, W, H), dtype=torch.uint8, device="cuda"))
    res_maps = L.ResidualMaps()
    res_maps.rgb, res_maps.depth, res_maps.alpha = (r.images[k].data_ptr() for k in ("rgb", "depth", "alpha"))
    res_maps.cosine, res_maps.obs_rgb, res_maps.obs_depth = (obs[k].data_ptr() for k in ("cosine", "obs_rgb",
                                                                                          "obs_depth"))
    res_opts = L.residual_opts()
    L.profile_enable((1 << L.K_NUM) - 1)
    for _ in range(10):
        step()
    # the residual kernels are short: a queued delay keeps the device busy
    # while the host enqueues them, so their events time the kernels alone
    torch.cuda._sleep(20_000_000)
    for _ in range(10):
        L.tracking_residual(V, W, H, res_opts, res_maps, res_out["R"], res_out["sigma"], res_out["dynamic"],
                            res_out["xi"], res_out["work"])
    torch.cuda.synchronize()
    names = ["project", "sort", "blend_fwd", "blend_bwd", "project_bwd", "decode", "decode_bwd", "residual"]
    br = {}
    for c, nm in enumerate(names):
        t, n = L.profile_read(c)
        if n:
            br[nm] = roofline_entry(t / n, ab[nm], ops.get(nm, {}))
    L.profile_enable(0)
    br["blend_fwd"]["note"] = "includes the fused L1 residual gradient of the step"
    br["residual"]["note"] = "tracking residual + uncertainty on the step's maps (not part of the timed step)"
    br.update(time_mapping_kernels(r, V, H, W, wl["seed"]))
    res["kernels"] = br
    res["config"]["pixel_evaluations"] = evals
    if args.serve_seconds > 0:
        res["serving"] = serving_c5(warmup_s=2.0, measure_s=args.serve_seconds)
    if not args.no_cpu_baseline:
        g_rng = np.random.default_rng(7)  # seeded upstream gradient of the frame's shape
        G = {"rgb": g_rng.normal(size=(3, H, W)), "depth": g_rng.normal(size=(H, W)),
             "feat": g_rng.normal(size=(16, H, W)), "alpha": g_rng.normal(size=(H, W))}
        res["cpu_baseline"] = cpu_baseline(sc, cam, G)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
