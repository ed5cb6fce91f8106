"""Per-tile depth ordering (tile-based rasterisation the paper follows, Sec. 3.1).

Test infrastructure (see the package docstring).

Every visible Gaussian is listed in each tile of its rectangle; each tile's
list is ordered by float32 camera depth, ties by ascending Gaussian index.
Written with numpy's lexsort, not a radix sort.
"""
from __future__ import annotations

import numpy as np


def bin_and_sort(rect: np.ndarray, z32: np.ndarray, visible: np.ndarray, tiles_x: int,
                 tiles_y: int, view: int = 0):
    """Return (tile_ids, gauss_ids, ranges) with tile_ids/gauss_ids of length
    I in sorted order and ranges (tiles_x*tiles_y, 2) = [start, end) per tile
    (row-major tile index ty*tiles_x + tx)."""
    tiles, gids = [], []
    for n in np.flatnonzero(visible):
        tx0, tx1, ty0, ty1 = rect[n]
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                tiles.append(ty * tiles_x + tx)
                gids.append(n)
    tiles = np.asarray(tiles, dtype=np.int64)
    gids = np.asarray(gids, dtype=np.int64)
    if tiles.size:
        order = np.lexsort((gids, z32[gids], tiles))
        tiles, gids = tiles[order], gids[order]
    nt = tiles_x * tiles_y
    starts = np.searchsorted(tiles, np.arange(nt), side="left")
    ends = np.searchsorted(tiles, np.arange(nt), side="right")
    ranges = np.stack([starts, ends], 1).astype(np.int64)
    return tiles, gids, ranges
