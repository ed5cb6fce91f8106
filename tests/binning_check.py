"""Tile-list checks by integer arithmetic (test infrastructure).

Two checks of the binning step of the tile rasteriser (Sec. 3.1):

* self-consistency: the tile rectangles, the sorted (tile, depth, index)
  pairs and the per-tile ranges are re-derived from the kernels' own float32
  footprint values (u, v, r_x, r_y, depth key) with integer arithmetic and
  numpy's lexsort, and must equal the kernels' lists bit for bit, with no
  exclusion;
* cross-precision: the kernels' lists against the FP64 oracle's, where only
  Gaussians inside a stated band of a threshold (a rectangle edge, a depth tie
  within a few float32 ulps) may differ; their number is reported.

Everything here is plain numpy on arrays; nothing imports the product path.
"""
from __future__ import annotations

import numpy as np


def rects_from_footprint(u, v, rx, ry, tiles_x, tiles_y, tile=16):
    """Tile rectangle [tx0, tx1, ty0, ty1] of every entry from its centre and
    whole-pixel radii (float32 values, exact in float64): tx0 = max(0,
    floor((floor(u) - r_x) / T)), tx1 = min(TX - 1, floor((floor(u) + r_x) / T)),
    likewise in y. tiles_x / tiles_y may be per-entry arrays. An entry with a
    negative radius (culled before the footprint) or an empty rectangle is not
    listed. Returns (rect (N,4) int64, listed (N,) bool)."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    rx = np.asarray(rx, np.float64)
    ry = np.asarray(ry, np.float64)
    staged = (rx >= 0) & (ry >= 0) & np.isfinite(u) & np.isfinite(v)
    iu = np.floor(np.where(staged, u, 0.0))
    iv = np.floor(np.where(staged, v, 0.0))
    rxs = np.where(staged, rx, 0.0)
    rys = np.where(staged, ry, 0.0)
    tx0 = np.maximum(0.0, np.floor((iu - rxs) / tile))
    tx1 = np.minimum(np.asarray(tiles_x, np.float64) - 1.0, np.floor((iu + rxs) / tile))
    ty0 = np.maximum(0.0, np.floor((iv - rys) / tile))
    ty1 = np.minimum(np.asarray(tiles_y, np.float64) - 1.0, np.floor((iv + rys) / tile))
    listed = staged & (tx0 <= tx1) & (ty0 <= ty1)
    rect = np.stack([tx0, tx1, ty0, ty1], 1).astype(np.int64)
    return rect, listed


def lists_from_rects(rect, listed, dkey, view_of, tile_base, tiles_x, n_tiles):
    """Sorted pairs of every listed entry over its rectangle, ordered by
    (global tile, depth key, entry index) with lexsort; ranges [start, end)
    per global tile. dkey: uint32 float bits (ascending = ascending positive
    depth). Returns (tile (I,), gid (I,), ranges (n_tiles, 2)), int64."""
    g = np.flatnonzero(listed)
    w = rect[g, 1] - rect[g, 0] + 1
    h = rect[g, 3] - rect[g, 2] + 1
    cnt = w * h
    total = int(cnt.sum())
    gids = np.repeat(g, cnt)
    k = np.arange(total, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    wr = np.repeat(w, cnt)
    tx = np.repeat(rect[g, 0], cnt) + k % wr
    ty = np.repeat(rect[g, 2], cnt) + k // wr
    vv = np.asarray(view_of)[gids]
    tile = np.asarray(tile_base, np.int64)[vv] + ty * np.asarray(tiles_x, np.int64)[vv] + tx
    keys = np.asarray(dkey).astype(np.uint32)[gids].astype(np.int64)
    order = np.lexsort((gids, keys, tile))
    tile, gids = tile[order], gids[order]
    t = np.arange(n_tiles)
    ranges = np.stack([np.searchsorted(tile, t, "left"), np.searchsorted(tile, t, "right")], 1)
    return tile.astype(np.int64), gids.astype(np.int64), ranges.astype(np.int64)


def self_consistency(st, views, n, tile=16):
    """Compare a context's binning with its re-derivation from its own
    footprint values. st: dict of numpy arrays geom (V*n, 8), radius (V*n, 2),
    dkey (V*n,) uint32, ntiles (V*n,), rect (V*n, 4), pair_tile (I,),
    pair_gauss (I,), ranges (T, 2), n_isect, n_visible. views: list of
    (width, height). Returns a dict of mismatch counts (all zero when the
    binning is exact) and sizes."""
    V = len(views)
    TX = np.array([-(-w // tile) for w, _ in views], np.int64)
    TY = np.array([-(-h // tile) for _, h in views], np.int64)
    tile_base = np.concatenate([[0], np.cumsum(TX * TY)[:-1]]).astype(np.int64)
    n_tiles = int((TX * TY).sum())
    view_of = np.repeat(np.arange(V), n)
    geom, rad = st["geom"], st["radius"]
    rect, listed = rects_from_footprint(geom[:, 0], geom[:, 1], rad[:, 0], rad[:, 1], TX[view_of], TY[view_of],
                                        tile)
    ntl = np.asarray(st["ntiles"]).astype(np.int64)
    dkey = np.asarray(st["dkey"]).astype(np.uint32)
    grect = np.asarray(st["rect"]).astype(np.int64)
    area = (rect[:, 1] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 2] + 1)
    out = dict(n_listed=int(listed.sum()))
    out["listed_mismatch"] = int(((ntl > 0) != listed).sum())
    out["rect_mismatch"] = int((grect[listed] != rect[listed]).any(1).sum())
    out["ntiles_mismatch"] = int((ntl[listed] != area[listed]).sum())
    # a listed entry's key is a positive finite float32 depth; an unlisted one is all ones
    kf = dkey[listed].view(np.float32)
    out["key_invalid"] = int((~np.isfinite(kf) | (kf <= 0)).sum()) + int((dkey[~listed] != 0xFFFFFFFF).sum())
    out["count_mismatch"] = int(int(st["n_isect"]) != int(area[listed].sum())) + \
        int(int(st["n_visible"]) != int(listed.sum()))
    tile_e, gid_e, rng_e = lists_from_rects(rect, listed, dkey, view_of, tile_base, TX, n_tiles)
    I = len(tile_e)
    pt = np.asarray(st["pair_tile"]).astype(np.int64)[:I]
    pg = np.asarray(st["pair_gauss"]).astype(np.int64)[:I]
    out["n_isect"] = I
    out["pair_tile_mismatch"] = int((pt != tile_e).sum()) if len(pt) == I else I
    out["pair_gauss_mismatch"] = int((pg != gid_e).sum()) if len(pg) == I else I
    out["range_mismatch"] = int((np.asarray(st["ranges"]).astype(np.int64) != rng_e).any(1).sum())
    return out


def rect_band(u, v, sx, sy, tiles_x, tiles_y, eps_u=1e-3, eps_s=1e-4, tile=16):
    """Entries whose tile rectangle (or listing) changes when the centre moves
    by eps_u pixels or the unrounded radius by eps_s * max(1, radius): where a
    float32 and a float64 evaluation may take the integer decision
    differently. Returns a boolean mask."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    sx = np.asarray(sx, np.float64)
    sy = np.asarray(sy, np.float64)
    base, lb = rects_from_footprint(u, v, np.ceil(sx), np.ceil(sy), tiles_x, tiles_y, tile)
    flag = np.zeros(len(u), bool)
    for du in (-eps_u, eps_u):
        for dv in (-eps_u, eps_u):
            for ds in (-eps_s, eps_s):
                r, l = rects_from_footprint(u + du, v + dv, np.ceil(sx + ds * np.maximum(1.0, sx)),
                                            np.ceil(sy + ds * np.maximum(1.0, sy)), tiles_x, tiles_y, tile)
                flag |= (l != lb) | (lb & l & (r != base).any(1))
    return flag


def tie_band(gids, ranges, z32, ulps):
    """Entries with a neighbour in some tile list whose float32 depth is
    within `ulps` float32 ulps: their relative order may be taken either way
    by two evaluations of the depth that round differently."""
    z = np.asarray(z32, np.float32)
    out = set()
    for s, e in ranges:
        if e - s < 2:
            continue
        g = gids[s:e]
        zz = z[g]
        gap = (zz[1:].astype(np.float64) - zz[:-1]) / np.spacing(zz[:-1]).astype(np.float64)
        for j in np.flatnonzero(gap <= ulps):
            out.add(int(g[j]))
            out.add(int(g[j + 1]))
    return out


def compare_lists(ref_gids, ref_ranges, gpu_gids, gpu_ranges, flagged):
    """Number of tiles whose lists differ once the flagged entries are
    removed from both sides."""
    flagged = np.fromiter(flagged, np.int64) if not isinstance(flagged, np.ndarray) else flagged
    fset = np.zeros(int(max(ref_gids.max(initial=0), gpu_gids.max(initial=0))) + 1, bool)
    fset[flagged[flagged < len(fset)]] = True
    bad = 0
    for t in range(ref_ranges.shape[0]):
        s, e = ref_ranges[t]
        a = ref_gids[s:e]
        a = a[~fset[a]]
        gs, ge = gpu_ranges[t]
        b = gpu_gids[gs:ge]
        b = b[~fset[b]]
        if len(a) != len(b) or not np.array_equal(a, b):
            bad += 1
    return bad
