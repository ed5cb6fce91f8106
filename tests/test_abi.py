"""The C ABI on the host: the library loads, exports every declared symbol,
and rejects bad arguments before launching anything (no GPU needed)."""
import ctypes as C

import numpy as np
import pytest

import synth
from paper_2505_22335_amd import _lib as L


def test_every_declared_symbol_is_exported():
    names = L.declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L.lib, n), n
    assert L.lib.asgs_abi_version() == 1


def test_status_strings():
    for s in range(6):
        assert L.lib.asgs_status_string(s)
    assert L.lib.asgs_last_error() is not None


def test_ctx_size_grows_with_capacity_and_views():
    cam = synth.camera_c2()
    o = L.make_opts(16)
    b0 = L.render_ctx_size([cam], 200_000, o, 0)
    b1 = L.render_ctx_size([cam], 200_000, o, 1_000_000)
    b2 = L.render_ctx_size([cam, cam], 200_000, o, 1_000_000)
    assert b0 < b1 < b2
    assert b1 - b0 >= 1_000_000 * (6 * 4 + 26 * 4)  # pair arrays + gradient slots


@pytest.mark.parametrize("field,value,status", [
    ("n_feat", 3, L.E_UNSUPPORTED), ("tile", 8, L.E_UNSUPPORTED), ("alpha_min", 0.0, L.E_INVALID),
    ("T_min", 2.0, L.E_INVALID), ("znear", -1.0, L.E_INVALID), ("extent_mode", 2, L.E_INVALID)])
def test_bad_options_rejected(field, value, status):
    o = L.make_opts(16)
    setattr(o, field, value)
    with pytest.raises(L.AsgsError) as ei:
        L.render_ctx_size([synth.camera_c2()], 100, o, 10)
    assert ei.value.status == status


def test_bad_cameras_rejected():
    cam = synth.camera_c2()
    bad = synth.Camera(0, 480, 525.0, 525.0, 319.5, 239.5, cam.T_wc)
    with pytest.raises(L.AsgsError):
        L.render_ctx_size([bad], 100, L.make_opts(16), 10)
    T = cam.T_wc.copy()
    T[0, 3] = np.nan
    with pytest.raises(L.AsgsError) as ei:
        L.render_ctx_size([cam.copy_with(T)], 100, L.make_opts(16), 10)
    assert "non-finite" in str(ei.value)
    with pytest.raises(L.AsgsError):
        L.render_ctx_size([cam] * 65, 100, L.make_opts(16), 10)


def test_null_and_misaligned_pointers_rejected_before_launch():
    cam = L.make_cameras([synth.camera_c1()])
    o = L.make_opts(0)
    g = L.Gaussians()
    g.n = 10
    out = L.Images()
    st = L.lib.asgs_render_forward(cam, 1, C.byref(g), C.byref(o), C.byref(out), None, 0, None)
    assert st == L.E_INVALID
    buf = (C.c_float * 64)()
    base = C.addressof(buf)
    g.mean = g.scale = g.rot = g.opacity = g.rgb = base + 4  # misaligned
    out.rgb = out.depth = out.alpha = base
    st = L.lib.asgs_render_forward(cam, 1, C.byref(g), C.byref(o), C.byref(out), base, 64, None)
    assert st == L.E_INVALID and b"aligned" in L.lib.asgs_last_error()


def test_small_context_reports_required_bytes():
    cam = L.make_cameras([synth.camera_c1()])
    o = L.make_opts(0)
    buf = (C.c_float * 64)()
    base = (C.addressof(buf) + 255) // 256 * 256 if False else C.addressof(buf)
    g = L.Gaussians()
    g.n = 10
    g.mean = g.scale = g.rot = g.opacity = g.rgb = base
    out = L.Images()
    out.rgb = out.depth = out.alpha = base
    st = L.lib.asgs_render_forward(cam, 1, C.byref(g), C.byref(o), C.byref(out), 256, 64, None)
    assert st == L.E_WORKSPACE and b"needs at least" in L.lib.asgs_last_error()


def test_decoder_parameter_count():
    d = L.make_decoder(1000, 10, 16)
    n = L.decode_param_count(d)
    per_head = lambda m: 32 * 35 + 32 + 10 * m * 32 + 10 * m
    assert n == sum(per_head(m) for m in (1, 3, 3, 4, 16))
    d0 = L.make_decoder(1000, 10, 0)
    assert L.decode_param_count(d0) == sum(per_head(m) for m in (1, 3, 3, 4))
    with pytest.raises(L.AsgsError):
        L.decode_param_count(L.make_decoder(1000, 17, 16))
    # per-view camera-centre partials: one row of 3 floats per 256 anchors and view
    big = L.make_decoder(100_000, 10, 16)
    assert L.decode_workspace_size(big, 2) > L.decode_workspace_size(big, 1) >= L.decode_workspace_size(d, 1)


def test_decoder_input_widths():
    """in_dim 35 (or 0), 36 and 38 are accepted; each extra input column adds
    one first-layer weight per hidden unit of every present head (5 heads
    with the feature head, 4 without); other widths are not built."""
    for nf, heads in ((16, 5), (0, 4)):
        base = L.decode_param_count(L.make_decoder(100, 10, nf, in_dim=35))
        assert L.decode_param_count(L.make_decoder(100, 10, nf, in_dim=0)) == base
        assert L.decode_param_count(L.make_decoder(100, 10, nf, in_dim=36)) == base + 32 * heads
        assert L.decode_param_count(L.make_decoder(100, 10, nf, in_dim=38)) == base + 3 * 32 * heads
    for bad in (37, 34, 39, 64):
        with pytest.raises(L.AsgsError) as ei:
            L.decode_param_count(L.make_decoder(100, 10, 16, in_dim=bad))
        assert ei.value.status == L.E_UNSUPPORTED


def test_pack_params_layout_round_trip():
    """Per head: W1's first 35 columns, b1, W2, b2, then W1's extra columns;
    unpack inverts it for every input width."""
    import torch
    from paper_2505_22335_amd.core import pack_params, unpack_params
    for in_dim in (35, 36, 38):
        w = synth.anchor_weights(np.random.default_rng(in_dim), 3, in_dim=in_dim, n_feat=16)
        flat = pack_params(w, 3, 16, device="cpu")
        assert flat.numel() == L.decode_param_count(L.make_decoder(10, 3, 16, in_dim=in_dim))
        W1 = w["opacity"]["W1"]
        assert torch.equal(flat[:35], torch.as_tensor(W1[0, :35]))
        o = 32 * 35 + 32 + 3 * 32 + 3
        assert torch.equal(flat[o:o + (in_dim - 35)], torch.as_tensor(W1[0, 35:]))
        back = unpack_params(flat, 3, 16, in_dim)
        for h in w:
            for key in w[h]:
                assert np.array_equal(back[h][key].numpy(), w[h][key]), (in_dim, h, key)


def test_bad_frame_time_rejected():
    cam = synth.camera_c2()
    bad = synth.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.T_wc, t=float("inf"))
    with pytest.raises(L.AsgsError) as ei:
        L.render_ctx_size([bad], 100, L.make_opts(16), 10)
    assert "frame time" in str(ei.value)


def test_mapping_and_uncertainty_host_checks():
    """Size queries and argument checks of the mapping-loss, mean-scale and
    uncertainty calls (host side, nothing launched)."""
    b = L.mapping_work_size(2, 640, 480)
    assert b >= 2 * 9 * 640 * 480 * 4
    with pytest.raises(L.AsgsError) as ei:
        L.mapping_work_size(0, 640, 480)
    assert ei.value.status == L.E_INVALID
    o = L.mapping_opts()
    assert abs(o.lam - 0.8) < 1e-7 and abs(o.lam1 - 0.6) < 1e-7 and o.lam2 == 1.0 and abs(o.lam4 - 0.01) < 1e-9
    maps = L.MappingMaps()
    st = L.lib.asgs_mapping_loss(1, 8, 8, C.byref(o), C.byref(maps), None, None, None, None, None, 0, None)
    assert st == L.E_INVALID and b"missing" in L.lib.asgs_last_error()
    assert L.mean_scale_work_size() > 0
    u = L.uncertainty_mlp(384, 34, 46)
    assert L.uncertainty_param_count(u) == 128 * 384 + 257
    assert L.uncertainty_workspace_size(u, 1, 640, 480) > 34 * 46 * 128 * 4
    for bad, status in ((L.uncertainty_mlp(20, 34, 46), L.E_UNSUPPORTED), (L.uncertainty_mlp(384, 0, 46), L.E_INVALID),
                        (L.uncertainty_mlp(384, 34, 46, sigma_min=0.0), L.E_INVALID)):
        with pytest.raises(L.AsgsError) as ei:
            L.uncertainty_param_count(bad)
        assert ei.value.status == status
