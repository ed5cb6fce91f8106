"""GPU: one training step (decode, render forward, L1 loss gradient, render
backward, decoder backward) captured into a HIP graph replays bitwise equal to
the step launched kernel by kernel, on several replays with eager work and
synchronisations in between."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2505_22335_amd.pipeline import AnchorRenderer, anchors_to_device


def test_graph_replay_equals_eager():
    sc, cam, _ = synth.c2("shell", 2000, seed=12)
    log("case graph replay")
    r = AnchorRenderer(anchors_to_device(sc), [cam])
    r.fit()
    rng = np.random.default_rng(3)
    tgt = {k: torch.as_tensor(rng.uniform(size=s), dtype=torch.float32).cuda()
           for k, s in (("rgb", (1, 3, 480, 640)), ("depth", (1, 480, 640)), ("feat", (1, 16, 480, 640)),
                        ("alpha", (1, 480, 640)))}
    dimg = {k: torch.empty_like(v) for k, v in tgt.items()}
    out = {}

    def step():
        img = r.forward()
        for k in dimg:
            torch.sign(torch.sub(img[k], tgt[k]), out=dimg[k])
            dimg[k].mul_(1.0 / dimg[k].numel())
        g = r.backward(dimg)
        out.update(img=img, g=g)

    def snapshot():
        s = {"img_" + k: v.clone() for k, v in out["img"].items()}
        s.update({"d_" + k: out["g"]["d_" + k].clone() for k in ("xyz", "feat", "off", "params", "pose")})
        return s

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    ref = snapshot()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        got = snapshot()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (rep, k)
        # eager work between replays must not disturb the next replay
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    log("graph replays equal eager:", sorted(ref))
