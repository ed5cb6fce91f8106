"""The integer tile-list checker (tests/binning_check.py) against the oracle's
own binning, and its sensitivity to planted mistakes (CPU only)."""
import numpy as np

import oracle
import synth
from oracle.geometry import pose_cw
from tests import binning_check as BC


def _proj(sc, cam, opts):
    g = oracle.gaussians_from_plain(sc)
    R, t = pose_cw(np.asarray(cam.T_wc, np.float64))
    return oracle.project(g["mean"], g["scale"], g["rot"], g["opacity"], R, t, cam.width, cam.height,
                          cam.fx, cam.fy, cam.cx, cam.cy, opts)


def _state_from_oracle(projs, cams, n):
    """A context-like state assembled from oracle projections of several views
    (view v's Gaussians at v*n + i), lists from the oracle's own binning."""
    geom, rad, dkey, ntl, rect, tiles, gids = [], [], [], [], [], [], []
    base = 0
    for v, (p, cam) in enumerate(zip(projs, cams)):
        TX, TY = p["tiles_xy"]
        u = p["u"].detach().numpy().astype(np.float32)
        vv = p["v"].detach().numpy().astype(np.float32)
        g = np.zeros((n, 8), np.float32)
        g[:, 0], g[:, 1] = u, vv
        r = p["radius"].astype(np.float32).copy()
        front = p["z"].detach().numpy() > 0.2
        r[~front] = -1.0
        k = p["z32"].view(np.uint32).copy()
        k[~p["visible"]] = 0xFFFFFFFF
        geom.append(g)
        rad.append(r)
        dkey.append(k)
        ntl.append(p["ntiles"])
        rect.append(np.where(p["visible"][:, None], p["rect"], np.array([1, 0, 1, 0])))
        t, gi, _ = oracle.bin_and_sort(p["rect"], p["z32"], p["visible"], TX, TY)
        tiles.append(t + base)
        gids.append(gi + v * n)
        base += TX * TY
    tiles = np.concatenate(tiles)
    gids = np.concatenate(gids)
    o = np.argsort(tiles, kind="stable")  # per-view blocks are already tile-sorted
    tiles, gids = tiles[o], gids[o]
    T = np.arange(base)
    ranges = np.stack([np.searchsorted(tiles, T, "left"), np.searchsorted(tiles, T, "right")], 1)
    nt = np.concatenate(ntl)
    return dict(geom=np.concatenate(geom), radius=np.concatenate(rad), dkey=np.concatenate(dkey),
                ntiles=nt, rect=np.concatenate(rect), pair_tile=tiles, pair_gauss=gids, ranges=ranges,
                n_isect=int(nt.sum()), n_visible=int((nt > 0).sum()))


def _two_view_case():
    sc = synth.tiny_scene(11, 400, logs_mu=-2.6)
    base = np.eye(3, 4, dtype=np.float32)
    cams = [synth.Camera(70, 45, 60.0, 60.0, 34.5, 22.0, base),
            synth.Camera(70, 45, 60.0, 60.0, 34.5, 22.0, synth.perturb_pose(base, [0.05, -0.02, 0.0],
                                                                               [0.0, 0.03, 0.01]))]
    opts = oracle.RenderOpts(n_feat=0)
    projs = [_proj(sc, c, opts) for c in cams]
    return sc, cams, projs


def test_checker_reproduces_oracle_binning():
    """Rectangles from (u, v, r) and the lexsort lists equal the oracle's
    binning (enumeration of rectangles + lexsort) for two views."""
    sc, cams, projs = _two_view_case()
    st = _state_from_oracle(projs, cams, sc.n)
    res = BC.self_consistency(st, [(c.width, c.height) for c in cams], sc.n)
    assert res["n_isect"] > 1000
    for k, v in res.items():
        if k.endswith("mismatch") or k == "key_invalid":
            assert v == 0, (k, v)


def test_checker_catches_planted_mistakes():
    sc, cams, projs = _two_view_case()
    views = [(c.width, c.height) for c in cams]
    st = _state_from_oracle(projs, cams, sc.n)
    # two neighbours of one list swapped
    s2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    t = int(np.argmax(st["ranges"][:, 1] - st["ranges"][:, 0]))
    a = st["ranges"][t, 0]
    s2["pair_gauss"][[a, a + 1]] = s2["pair_gauss"][[a + 1, a]]
    assert BC.self_consistency(s2, views, sc.n)["pair_gauss_mismatch"] == 2
    # a rectangle one tile too wide
    s3 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    j = int(np.flatnonzero(st["ntiles"] > 0)[0])
    s3["rect"][j, 1] += 1
    assert BC.self_consistency(s3, views, sc.n)["rect_mismatch"] == 1
    # a range end moved by one
    s4 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    s4["ranges"][t, 1] -= 1
    assert BC.self_consistency(s4, views, sc.n)["range_mismatch"] == 1
    # a depth key that no longer orders the list (a flipped low bit changes the order of a near tie
    # only if one exists; a key of the wrong entry always does)
    s5 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    g0, g1 = s5["pair_gauss"][a], s5["pair_gauss"][a + 1]
    s5["dkey"][[g0, g1]] = s5["dkey"][[g1, g0]]
    r5 = BC.self_consistency(s5, views, sc.n)
    assert r5["pair_gauss_mismatch"] > 0 or s5["dkey"][g0] == s5["dkey"][g1]


def test_rect_band_flags_only_edge_cases():
    """A centre 2e-4 px below an integer whose floor decides a tile edge is
    flagged; the same Gaussian in the middle of its pixel is not."""
    TX, TY = 4, 4
    # u = 17.9998, r = 2: floor(u) - r is 15 (tile 0) or 16 (tile 1) within the band -> flagged;
    # u = 17.5: clear; u = 15.9998, r = 3: both floors keep the same tiles -> clear;
    # r = ceil(6.99995) is 7 or 8 within the band and 40 + r crosses 48 -> flagged
    u = np.array([17.9998, 17.5, 15.9998, 40.0])
    v = np.array([8.5, 8.5, 8.5, 8.5])
    sx = np.array([1.5, 1.5, 2.5, 6.99995])
    sy = np.array([0.5, 0.5, 0.5, 0.5])
    f = BC.rect_band(u, v, sx, sy, TX, TY, eps_u=1e-3, eps_s=1e-4)
    assert f.tolist() == [True, False, False, True]


def test_tie_band():
    z = np.array([1.0, np.nextafter(np.float32(1.0), np.float32(2.0)), 1.5, 2.0], np.float32)
    gids = np.array([0, 1, 2, 3])
    ranges = np.array([[0, 4]])
    assert BC.tie_band(gids, ranges, z, 4) == {0, 1}
    assert BC.tie_band(gids, ranges, z, 0.5) == set()
    assert BC.compare_lists(gids, ranges, np.array([1, 0, 2, 3]), ranges, np.array([0, 1])) == 0
    assert BC.compare_lists(gids, ranges, np.array([0, 1, 3, 2]), ranges, np.array([0, 1])) == 1
