"""GPU: the allocation-free L1 residual entry point (asgs_l1_loss_noalloc)
against asgs_l1_loss with a caller workspace, through the C ABI: two calls in
a row, the second with fewer views and a smaller image (the scratch array
keeps the first call's partials, which the second must not read), plus a
third call over the maximum view count of the scratch and one beyond it."""
import ctypes as C

import pytest
import torch

from tests.gpu_util import log

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2505_22335_amd import _lib as L
    from paper_2505_22335_amd.core import l1_targets


def _case(V, H, W, nf, seed, use_weight):
    g = torch.Generator().manual_seed(seed)
    mk = lambda *s: torch.rand(*s, generator=g).cuda()
    maps = {"rgb": mk(V, 3, H, W), "depth": mk(V, H, W), "alpha": mk(V, H, W)}
    tgt = {"rgb": mk(V, 3, H, W), "depth": mk(V, H, W), "alpha": mk(V, H, W)}
    if nf:
        maps["feat"] = mk(V, nf, H, W)
        tgt["feat"] = mk(V, nf, H, W)
    weight = mk(H, W) if use_weight else None
    scale = {"rgb": 0.5, "depth": 2.0, "feat": 0.25, "alpha": 3.0}
    return maps, tgt, weight, scale


def _run(fn_noalloc, V, H, W, nf, seed, use_weight):
    maps, tgt, weight, scale = _case(V, H, W, nf, seed, use_weight)
    t = l1_targets(tgt, scale, weight)
    outs = []
    for noalloc in (False, True):
        grad = {k: torch.full_like(v, 7.0) for k, v in maps.items()}
        loss = torch.full((V,), -1.0, device="cuda")
        if noalloc:
            fn_noalloc(V, W, H, nf, L.make_images(maps), t, L.make_images(grad), loss)
        else:
            work = torch.empty(L.l1_loss_work_size(V), dtype=torch.uint8, device="cuda")
            L.l1_loss(V, W, H, nf, L.make_images(maps), t, L.make_images(grad), loss, work)
        torch.cuda.synchronize()
        outs.append((grad, loss))
    (g0, l0), (g1, l1) = outs
    for k in g0:
        assert torch.equal(g0[k], g1[k]), k
    # same kernels, same fixed-order sums: the loss is bitwise equal
    assert torch.equal(l0, l1), (l0.tolist(), l1.tolist())
    log("noalloc", V, H, W, nf, "loss", l1.tolist()[:4])


def test_noalloc_l1_equals_workspace_version_twice():
    _run(L.l1_loss_noalloc, 3, 48, 64, 16, 1, True)
    _run(L.l1_loss_noalloc, 1, 23, 37, 0, 2, False)  # second call: smaller input
    _run(L.l1_loss_noalloc, L.MAX_VIEWS, 8, 12, 16, 3, True)  # the scratch's maximum


def test_noalloc_l1_rejects_more_views_than_its_scratch():
    maps, tgt, weight, scale = _case(1, 8, 8, 0, 4, False)
    t = l1_targets(tgt, scale, weight)
    loss = torch.empty(1, device="cuda")
    st = L.lib.asgs_l1_loss_noalloc(L.MAX_VIEWS + 1, 8, 8, 0, C.byref(L.make_images(maps)), C.byref(t),
                                    C.byref(L.make_images(maps)), loss.data_ptr(), L._stream())
    assert st == L.E_UNSUPPORTED
    assert b"at most" in L.lib.asgs_last_error()
