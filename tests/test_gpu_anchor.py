"""GPU: the probabilistic anchor update (asgs_anchor_update; Sec. 3.3 Eq. 7)
against the FP64 oracle, through the C ABI. Probabilities within 1e-6
relative (a handful of FP32 operations), keep flags and their count bit for
bit except where the oracle's result sits within 1e-6 of the pruning level."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2505_22335_amd import _lib as L


@pytest.mark.parametrize("n,opts", [(1, {}), (1000, dict(prior=0.3)), (1_000_003, dict(prior=0.6, p_min=0.12,
                                                                                   p_max=0.97, prune_below=0.2))])
def test_anchor_update_matches_oracle(n, opts):
    log("case anchor update", n, opts)
    rng = np.random.default_rng(n)
    pp = rng.uniform(0.02, 0.98, n).astype(np.float32)
    po = rng.uniform(0.02, 0.98, n).astype(np.float32)
    ref, keep_ref = oracle.anchor_update(pp, po, **opts)
    p = torch.as_tensor(pp).cuda()
    keep = torch.empty(n, dtype=torch.uint8, device="cuda")
    n_keep = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    L.anchor_update(torch.as_tensor(po).cuda(), p, keep, n_keep, **opts)
    torch.cuda.synchronize()
    got = p.cpu().numpy().astype(np.float64)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    band = np.abs(ref - opts.get("prune_below", 0.0)) <= 1e-6
    mism = int(((keep.cpu().numpy() != 0) != keep_ref)[~band].sum())
    log("anchor update rel err %.2e keep mismatches %d band %d kept %d" % (e, mism, int(band.sum()),
                                                                         int(n_keep.item())))
    assert e <= 1e-6 and mism == 0
    assert abs(int(n_keep.item()) - int(keep_ref.sum())) <= int(band.sum())
    assert int(n_keep.item()) == int(keep.sum().item())
