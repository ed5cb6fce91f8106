"""Pins for the oracle's anchor decoder (Sec. 3.3, Eq. 8 and Eq. 9).

Special cases with closed forms: zero second layers give act(b2); selector
first layers expose the input order, the sign of the view direction and the
hidden activation of each head; means are anchor + scaled offset; the
bfloat16 mode stays within the rounding bound of its operands.
"""
import math

import numpy as np
import torch

import synth
from oracle import decode, HEAD_ORDER

F64 = torch.float64


def _tens(sc):
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    w = {h: {k: t(v) for k, v in d.items()} for h, d in sc.weights.items()}
    return t(sc.xyz.T), t(sc.feat), t(sc.off.T), w


def _sig(x):
    return 1 / (1 + np.exp(-x))


def test_zero_second_layer_gives_bias_activations():
    sc = synth.tiny_anchor_scene(1, 7, k=3, n_feat=5)
    xyz, feat, off, w = _tens(sc)
    for h in w:
        w[h]["W2"] = torch.zeros_like(w[h]["W2"])
    g = decode(xyz, feat, off, w, torch.tensor([0.1, -0.2, 0.3], dtype=F64), sc.k, sc.l_o, sc.l_s)
    k = sc.k
    b = {h: sc.weights[h]["b2"].astype(np.float64).reshape(k, -1) for h in sc.weights}
    A = sc.n_anchors
    np.testing.assert_allclose(g["opacity"].numpy(), np.tile(_sig(b["opacity"][:, 0]), A), rtol=1e-12)
    np.testing.assert_allclose(g["rgb"].numpy(), np.tile(_sig(b["rgb"]), (A, 1)), rtol=1e-12)
    np.testing.assert_allclose(g["scale"].numpy(), np.tile(sc.l_s * _sig(b["scale"]), (A, 1)), rtol=1e-12)
    np.testing.assert_allclose(g["rot"].numpy(), np.tile(b["rot"], (A, 1)), rtol=1e-12)
    np.testing.assert_allclose(g["feat"].numpy(), np.tile(b["feat"], (A, 1)), rtol=1e-12)
    np.testing.assert_allclose(g["mean"].numpy(),
                               np.repeat(sc.xyz.T.astype(np.float64), k, 0) + sc.l_o * sc.off.T, rtol=1e-12)


def test_selector_weights_expose_direction_and_activation():
    """First layer picks input column j (a feature, or a direction component);
    second layer averages the hidden units. Opacity = sigmoid(act(x_j) + b).
    The camera sits at the origin so the direction of anchor v is x_v/|x_v|."""
    k = 2
    xyz = torch.tensor([[3.0, 0.0, 0.0], [-2.0, 0.0, 0.0], [0.0, 0.0, 5.0]], dtype=F64)
    feat = torch.zeros((3, 32), dtype=F64)
    feat[:, 7] = torch.tensor([0.4, -0.9, 1.3])
    off = torch.zeros((3 * k, 3), dtype=F64)
    cases = [(32, "opacity"), (34, "opacity"), (7, "opacity"), (32, "feat"), (7, "feat")]
    for col, head in cases:
        w = {}
        for name, m, _ in HEAD_ORDER:
            mm = 2 if name == "feat" else m
            W1 = torch.zeros((32, 35), dtype=F64)
            W1[:, col] = 1.0
            w[name] = dict(W1=W1, b1=torch.zeros(32, dtype=F64),
                           W2=torch.full((k * mm, 32), 1.0 / 32, dtype=F64),
                           b2=torch.full((k * mm,), 0.25, dtype=F64))
        g = decode(xyz, feat, off, w, torch.zeros(3, dtype=F64), k)
        if col >= 32:
            x = (xyz / xyz.norm(dim=1, keepdim=True))[:, col - 32].numpy()
        else:
            x = feat[:, col].numpy()
        relu = np.maximum(x, 0)
        softplus = np.log1p(np.exp(x))
        if head == "opacity":
            np.testing.assert_allclose(g["opacity"].numpy(), np.repeat(_sig(relu + 0.25), k), rtol=1e-12)
        else:
            np.testing.assert_allclose(g["feat"].numpy(), np.repeat(softplus + 0.25, k)[:, None]
                                       * np.ones((1, 2)), rtol=1e-12)


def test_view_direction_follows_camera_centre():
    """Moving the camera along +x by 10 m flips the x direction of an anchor
    at the origin: a ReLU selector on direction-x then passes 0 instead of 1."""
    k = 1
    xyz = torch.zeros((1, 3), dtype=F64)
    feat = torch.zeros((1, 32), dtype=F64)
    off = torch.zeros((1, 3), dtype=F64)
    w = {}
    for name, m, _ in HEAD_ORDER[:4]:
        W1 = torch.zeros((32, 35), dtype=F64)
        W1[:, 32] = 1.0
        w[name] = dict(W1=W1, b1=torch.zeros(32, dtype=F64), W2=torch.full((m, 32), 1 / 32, dtype=F64),
                       b2=torch.zeros(m, dtype=F64))
    g_neg = decode(xyz, feat, off, w, torch.tensor([10.0, 0, 0], dtype=F64), k)   # dir = -x
    g_pos = decode(xyz, feat, off, w, torch.tensor([-10.0, 0, 0], dtype=F64), k)  # dir = +x
    assert abs(g_neg["opacity"].item() - 0.5) < 1e-15
    assert abs(g_pos["opacity"].item() - _sig(1.0)) < 1e-15


def test_bf16_mode_within_operand_rounding():
    sc = synth.tiny_anchor_scene(3, 40, k=10, n_feat=16)
    xyz, feat, off, w = _tens(sc)
    c = torch.tensor([0.0, 0.0, -0.5], dtype=F64)
    g64 = decode(xyz, feat, off, w, c, sc.k, sc.l_o, sc.l_s)
    g16 = decode(xyz, feat, off, w, c, sc.k, sc.l_o, sc.l_s, precision="bf16")
    for key in ("opacity", "rgb", "scale", "rot", "feat"):
        d = (g16[key] - g64[key]).abs().max().item()
        assert 0 < d < 2e-2, (key, d)
    assert torch.equal(g16["mean"], g64["mean"])


def test_bf16_mode_rounds_exactly_the_matrix_operands():
    """Hand-built rotation head (raw output, k = 1) where rounding each operand
    to bfloat16 moves the result by a distinct, known amount (u = 2^-7, the
    bfloat16 spacing in [1, 2)):
      hidden 0: anchor feature 1 + 0.75u (rounds to 1 + u), bias -0.375u
      hidden 1: first-layer weight 1 + 0.75u (rounds to 1 + u), bias -0.375u
      hidden 2: view-direction weight 1 + 0.375u (must stay exact), bias 0.25u
      hidden 3: pre-activation 1 + 0.25u (the hidden value rounds to 1)
      output 3: second-layer weight 1 + 0.75u (rounds to 1 + u)
      output 0: second-layer bias 1 + 2^-10 (must stay exact).
    Rounding a wrong operand, or missing one, changes at least one output."""
    u = 2.0 ** -7
    A, k = 1, 1
    xyz = torch.tensor([[2.0, 0.0, 0.0]], dtype=F64)   # unit view direction (1, 0, 0)
    c = torch.zeros(3, dtype=F64)
    feat = torch.zeros((1, 32), dtype=F64)
    feat[0, 0], feat[0, 1], feat[0, 3] = 1 + 0.75 * u, 1.0, 1.0
    off = torch.zeros((1, 3), dtype=F64)
    W = {}
    for name, m in (("opacity", 1), ("rgb", 3), ("scale", 3), ("rot", 4)):
        W[name] = dict(W1=torch.zeros((32, 35), dtype=F64), b1=torch.zeros(32, dtype=F64),
                       W2=torch.zeros((k * m, 32), dtype=F64), b2=torch.zeros(k * m, dtype=F64))
    w = W["rot"]
    w["W1"][0, 0], w["b1"][0] = 1.0, -0.375 * u
    w["W1"][1, 1], w["b1"][1] = 1 + 0.75 * u, -0.375 * u
    w["W1"][2, 32], w["b1"][2] = 1 + 0.375 * u, 0.25 * u
    w["W1"][3, 3], w["b1"][3] = 1.0, 0.25 * u
    w["W2"][0, 0], w["W2"][1, 1], w["W2"][2, 2], w["W2"][3, 3] = 1.0, 1.0, 1.0, 1 + 0.75 * u
    w["b2"][0] = 1 + 2.0 ** -10
    g16 = decode(xyz, feat, off, W, c, k, 1.0, 0.02, precision="bf16")
    g64 = decode(xyz, feat, off, W, c, k, 1.0, 0.02)
    expect16 = [2 + u + 2.0 ** -10, 1 + u, 1 + u, 1 + u]
    expect64 = [2 + 0.375 * u + 2.0 ** -10, 1 + 0.375 * u, 1 + 0.625 * u,
                (1 + 0.25 * u) * (1 + 0.75 * u)]
    assert g16["rot"][0].tolist() == expect16
    assert torch.allclose(g64["rot"][0], torch.tensor(expect64, dtype=F64), rtol=0, atol=1e-15)


def _widen(w, n_extra, rng=None):
    """Head weights with n_extra more first-layer columns (zero, or random)."""
    out = {}
    for h, d in w.items():
        e = torch.zeros((d["W1"].shape[0], n_extra), dtype=F64) if rng is None else \
            torch.as_tensor(rng.uniform(-0.3, 0.3, (d["W1"].shape[0], n_extra)))
        out[h] = dict(d, W1=torch.cat([d["W1"], e], 1))
    return out


def test_extra_inputs_with_zero_weights_reduce_to_base_decoder():
    """Distance and temporal columns with zero weights leave every output of
    the 35-input decoder unchanged (both precisions, any frame time)."""
    sc = synth.tiny_anchor_scene(3, 9, k=2, n_feat=16)
    xyz, feat, off, w = _tens(sc)
    c = torch.tensor([0.3, -0.1, -0.4], dtype=F64)
    for prec in ("fp64", "bf16"):
        base = decode(xyz, feat, off, w, c, sc.k, sc.l_o, sc.l_s, precision=prec)
        for n_extra in (1, 3):
            g = decode(xyz, feat, off, _widen(w, n_extra), c, sc.k, sc.l_o, sc.l_s, precision=prec, t=0.37)
            for key in base:
                assert torch.equal(g[key], base[key]), (prec, n_extra, key)


def test_distance_and_time_hand_case():
    """One anchor at (3, 4, 0) from a camera at the origin (distance 5), one
    opacity hidden unit fed by the distance (weight 1), sin(pi t) (weight 2)
    and cos(pi t) (weight 4) at t = 1/3: z = 5 + sqrt(3) + 2, and the second
    layer passes the unit through, so opacity = sigmoid(7 + sqrt(3))."""
    xyz = torch.tensor([[3.0, 4.0, 0.0]], dtype=F64)
    feat = torch.zeros((1, 32), dtype=F64)
    off = torch.zeros((1, 3), dtype=F64)
    w = {}
    for name, m, _ in HEAD_ORDER[:4]:
        W1 = torch.zeros((32, 38), dtype=F64)
        W2 = torch.zeros((m, 32), dtype=F64)
        if name == "opacity":
            W1[0, 35], W1[0, 36], W1[0, 37] = 1.0, 2.0, 4.0
            W2[0, 0] = 1.0
        w[name] = dict(W1=W1, b1=torch.zeros(32, dtype=F64), W2=W2, b2=torch.zeros(m, dtype=F64))
    g = decode(xyz, feat, off, w, torch.zeros(3, dtype=F64), 1, t=1.0 / 3.0)
    assert abs(float(g["opacity"][0]) - _sig(7.0 + math.sqrt(3.0))) < 1e-15
    # only the distance column: the unit reads 5 for any t
    w["opacity"]["W1"][0, 36:] = 0.0
    g = decode(xyz, feat, off, w, torch.zeros(3, dtype=F64), 1, t=0.8)
    assert abs(float(g["opacity"][0]) - _sig(5.0)) < 1e-15


def test_time_embedding_folds_into_bias_and_is_periodic():
    """At t = 1/2 the embedding is (1, 0): the 38-input decoder equals the
    36-input one with b1 + W1[:, 36]; at t = 1 it is (0, -1). Frames two
    time units apart share their embedding."""
    sc = synth.tiny_anchor_scene(4, 11, k=3, n_feat=16)
    xyz, feat, off, w = _tens(sc)
    rng = np.random.default_rng(5)
    w38 = _widen(w, 3, rng)
    c = torch.tensor([-0.2, 0.5, 0.1], dtype=F64)
    for t, col, sgn in ((0.5, 36, 1.0), (1.0, 37, -1.0)):
        w36 = {h: dict(d, W1=d["W1"][:, :36], b1=d["b1"] + sgn * d["W1"][:, col]) for h, d in w38.items()}
        g38 = decode(xyz, feat, off, w38, c, sc.k, sc.l_o, sc.l_s, t=t)
        g36 = decode(xyz, feat, off, w36, c, sc.k, sc.l_o, sc.l_s)
        for key in g36:
            assert (g38[key] - g36[key]).abs().max() < 1e-14, (t, key)
    g0 = decode(xyz, feat, off, w38, c, sc.k, sc.l_o, sc.l_s, t=0.3)
    g2 = decode(xyz, feat, off, w38, c, sc.k, sc.l_o, sc.l_s, t=2.3)
    for key in g0:
        assert (g0[key] - g2[key]).abs().max() < 1e-13
    with np.testing.assert_raises(ValueError):
        decode(xyz, feat, off, _widen(w, 2), c, sc.k)


def test_bf16_hidden_margin_hand_cases():
    """One opacity unit fed by one feature column (weight 1, bf16 exact):
    z = 1 + 2^-8 sits on the midpoint between the bfloat16 values 1 and
    1 + 2^-7 (margin 0); z = 1 is half a spacing (2^-8) from the midpoints,
    relative to the term sizes 1; z = 0 (ReLU zero) has no rounding risk."""
    from oracle import bf16_hidden_margin
    xyz = torch.tensor([[0.0, 0.0, 2.0], [0.0, 0.0, 3.0], [0.0, 0.0, 4.0]], dtype=F64)
    feat = torch.zeros((3, 32), dtype=F64)
    feat[:, 0] = torch.tensor([1.0 + 2.0 ** -8, 1.0, 0.0])
    w = {}
    for name, m, _ in HEAD_ORDER[:4]:
        W1 = torch.zeros((32, 35), dtype=F64)
        W1[0, 0] = 1.0
        w[name] = dict(W1=W1, b1=torch.zeros(32, dtype=F64), W2=torch.zeros((m, 32), dtype=F64),
                       b2=torch.zeros(m, dtype=F64))
    mg = bf16_hidden_margin(xyz, feat, w, torch.zeros(3, dtype=F64))
    # feature 1 + 2^-8 is itself rounded to bf16 (ties to even: 1.0) in layer 1, so z = 1
    assert mg["opacity"][0] == 2.0 ** -8 and mg["opacity"][1] == 2.0 ** -8
    assert np.isinf(mg["opacity"][2])
    # a bias moves z onto the midpoint: b1 = 2^-8 with the feature 1 gives
    # margin 0; alone (feature 0) z = 2^-8 is a bfloat16 value, half its
    # spacing 2^-15 from the midpoints, relative to |b1| = 2^-8
    w["opacity"]["b1"][0] = 2.0 ** -8
    mg = bf16_hidden_margin(xyz, feat, w, torch.zeros(3, dtype=F64))
    assert mg["opacity"][1] == 0.0 and mg["opacity"][2] == 2.0 ** -8


def test_bf16_flip_bound_hand_case():
    """A hidden unit on a bfloat16 rounding midpoint (z = 1 + 2^-8 with the
    feature 1 and b1 = 2^-8) may round to 1 or to 1 + 2^-7: the second layer
    (W2 = 1/2 on that unit, bf16 exact) then moves the pre-activation by
    2^-8, which the raw rotation head passes on and the sigmoid heads
    scale by at most 1/4 (the scale head by l_s / 4). Units off the band
    (z = 2^-8, margin 2^-8 relative to |b1|) contribute nothing. Both
    roundings are formed explicitly and their difference equals the bound."""
    from oracle import bf16_flip_bound
    xyz = torch.tensor([[0.0, 0.0, 2.0], [0.0, 0.0, 3.0]], dtype=F64)
    feat = torch.zeros((2, 32), dtype=F64)
    feat[:, 0] = torch.tensor([1.0, 0.0])
    k, l_s = 1, 0.02
    w = {}
    for name, m, _ in HEAD_ORDER[:4]:
        W1 = torch.zeros((32, 35), dtype=F64)
        W1[0, 0] = 1.0
        b1 = torch.zeros(32, dtype=F64)
        b1[0] = 2.0 ** -8
        W2 = torch.zeros((m, 32), dtype=F64)
        W2[:, 0] = 0.5
        w[name] = dict(W1=W1, b1=b1, W2=W2, b2=torch.zeros(m, dtype=F64))
    fb = bf16_flip_bound(xyz, feat, w, torch.zeros(3, dtype=F64), k, l_s=l_s)
    dy = 0.5 * ((1.0 + 2.0 ** -7) - 1.0)  # the two roundings of H through W2
    assert np.all(fb["rot"][0] == dy) and np.all(fb["rot"][1] == 0.0)
    assert np.all(fb["rgb"][0] == 0.25 * dy) and fb["opacity"][0, 0] == 0.25 * dy
    assert np.all(fb["scale"][0] == 0.25 * l_s * dy)
    # the sigmoid's largest slope bounds the change of the decoded value
    s = lambda y: 1.0 / (1.0 + np.exp(-y))
    assert abs(s(0.5 * (1.0 + 2.0 ** -7)) - s(0.5)) <= fb["opacity"][0, 0]
