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
    ("T_min", 2.0, L.E_INVALID), ("znear", -1.0, L.E_INVALID), ("reserved", 1, L.E_INVALID)])
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
