"""Throughput of the anchor-Gaussian hot path on one MI355X.

One step = decode (anchor MLPs) -> render forward (project, bin/sort, blend) ->
L1 loss gradient (PyTorch) -> render backward -> decode backward, for one batch
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


def algorithmic_bytes(I, nvis, N, A, P, nf=16):
    """Minimum bytes each kernel class must move (per launch), from the
    method's data: per intersection a 2D record (u,v,conic,opacity = 6
    floats) plus channels (rgb, depth, feature), per pixel the outputs or the
    upstream gradients, per Gaussian its parameters."""
    ch = 4 + nf
    rec = 4 * (6 + ch)
    return {
        "blend_fwd": I * rec + I * 4 + P * 4 * (ch + 1 + 2),
        "blend_bwd": I * rec + P * 4 * (ch + 1 + 2) + nvis * rec,
        "project": N * 4 * (3 + 3 + 4 + 1 + 3 + nf) + nvis * rec,
        "project_bwd": nvis * rec + N * 4 * (3 + 3 + 4 + 1) + N * 4 * (3 + 3 + 4 + 1 + 3 + nf),
        "decode": A * 4 * (3 + 32 + 30) + N * 4 * (3 + 3 + 4 + 1 + 3 + nf),
        "decode_bwd": N * 4 * (3 + 3 + 4 + 1 + 3 + nf) + A * 4 * 2 * (3 + 32 + 30),
    }


def cpu_baseline(sc, cam, G, budget_s=30.0):
    """The FP64 oracle's forward + backward of the same frame on the host."""
    import torch

    import oracle
    from oracle import RenderOpts
    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    oracle.render_scene(sc, cam, RenderOpts(n_feat=16), grad_out=G, pose_grad=True)
    dt = time.perf_counter() - t0
    mpix = cam.width * cam.height / 1e6
    return {"value": mpix / dt, "unit": "Mpix/s", "cores": threads, "kind": "oracle",
            "sample": f"one full {cam.width}x{cam.height} frame, forward+backward incl. decoder and pose "
                      f"({dt:.1f} s, torch CPU threads={threads})"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2s", choices=sorted(WORKLOADS))
    ap.add_argument("--views", type=int, default=1)
    ap.add_argument("--precision", type=int, default=0, help="decoder precision: 0 FP32, 1 BF16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--breakdown", action="store_true", help="also time every kernel class (untimed pass)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path is not sharded across GPUs in this build "
              "(see DESIGN.md, 'More than one GPU'). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2505_22335_amd import _lib as L
    from paper_2505_22335_amd.pipeline import AnchorRenderer, anchors_to_device

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
        img = r.forward()
        for k in dimg:  # L1 loss gradient, mean over each output
            torch.sign(torch.sub(img[k], tgt[k]), out=dimg[k])
            dimg[k].mul_(scale[k])
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
    L.profile_enable(1 << L.K_BLEND_BWD)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
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
        "data": "synthetic",
        "config": {"workload": wl["desc"] + f", {V} view(s), decoder {'FP32' if args.precision == 0 else 'BF16'}",
                   "anchors": A, "gaussians": N, "views": V, "width": W, "height": H, "n_feat": 16,
                   "intersections": I, "visible": nvis},
        "roofline": {"bound": "hbm", "kernel": "blend backward (k_blend_bwd)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_ms": round(dom_ms, 5), "launches": bb_n,
                     "algorithmic_bytes": int(ab["blend_bwd"])},
        "wall_s": round(wall, 3),
    }
    if args.breakdown:
        L.profile_enable((1 << L.K_NUM) - 1 if hasattr(L, "K_NUM") else 0x7F)
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        names = ["project", "sort", "blend_fwd", "blend_bwd", "project_bwd", "decode", "decode_bwd"]
        br = {}
        for c, nm in enumerate(names):
            t, n = L.profile_read(c)
            avg = t / max(n, 1)
            entry = {"avg_ms": round(avg, 5)}
            if nm in ab:
                entry["alg_GBs"] = round(ab[nm] / (avg * 1e-3) / 1e9, 1) if avg > 0 else None
            br[nm] = entry
        L.profile_enable(0)
        res["kernels"] = br
    if not args.no_cpu_baseline:
        g_rng = np.random.default_rng(7)  # seeded upstream gradient of the frame's shape
        G = {"rgb": g_rng.normal(size=(3, H, W)), "depth": g_rng.normal(size=(H, W)),
             "feat": g_rng.normal(size=(16, H, W)), "alpha": g_rng.normal(size=(H, W))}
        res["cpu_baseline"] = cpu_baseline(sc, cam, G)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
