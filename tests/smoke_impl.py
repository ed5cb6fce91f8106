"""One small decode -> render -> backward on cuda:0, checked against the oracle
(used by __graft_entry__.smoke)."""
from __future__ import annotations

import numpy as np


def run_smoke() -> None:
    import torch

    import oracle
    import synth
    from paper_2505_22335_amd.pipeline import AnchorRenderer, anchors_to_device
    from tests.gpu_util import GRAD_TOL, IMG_TOL, guard_mask, oracle_opts, rel_err, to_np, upstream

    assert torch.cuda.is_available(), "smoke needs a GPU"
    sc = synth.tiny_anchor_scene(11, 40, k=10, n_feat=16)
    cam = synth.Camera(80, 60, 60.0, 60.0, 39.5, 29.5,
                       synth.perturb_pose(np.eye(3, 4, dtype=np.float32), [0.02, 0.0, -0.1], [0.0, 0.02, 0.0]))
    ref = oracle.render_scene(sc, cam, oracle_opts(16), with_margins=True)
    keep = guard_mask(ref["margins"])
    G = upstream(1, cam.height, cam.width, 16)
    for k in G:
        G[k] = G[k] * keep
    r = AnchorRenderer(anchors_to_device(sc), [cam])
    r.fit()
    img = r.forward()
    grads = r.backward({k: torch.as_tensor(G[k][None]).cuda() for k in G})
    torch.cuda.synchronize()
    errs = {k: rel_err(to_np(img[k][0]), ref[k], keep) for k in ("rgb", "depth", "alpha", "feat")}
    _, gr = oracle.render_scene(sc, cam, oracle_opts(16), grad_out=G, pose_grad=True)
    errs["d_xyz"] = rel_err(to_np(grads["d_xyz"]), gr["anchor"]["xyz"])
    errs["d_feat"] = rel_err(to_np(grads["d_feat"]), gr["anchor"]["feat"])
    errs["d_pose"] = rel_err(to_np(grads["d_pose"][0]), gr["pose"])
    print("smoke errors:", {k: float("%.3g" % v) for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        tol = IMG_TOL if not k.startswith("d_") else GRAD_TOL
        assert v <= tol, (k, v)
    assert float(ref["alpha"].max()) > 0.3
