"""Screen-tile binning a tiled rasterizer must produce (test infrastructure only).

A visible Gaussian is listed in every tile that contains a pixel of its
inclusive pixel rectangle; tile id = ty * tiles_x + tx.  Each tile's list is
ordered by depth (Eq. 2 blends in depth order), equal depths by the Gaussian's
processing index.  The lists are laid out tile after tile; ranges[t] is the
[start, end) of tile t.  Written as plain enumeration plus a lexicographic sort.

reached_pairs gives the smaller set a tiled rasterizer has to keep: the tiles
in which a Gaussian's footprint ellipse at the cut level holds a pixel centre.
A renderer may list a Gaussian in any set of its rectangle's tiles between
the two without changing the image.
"""
from __future__ import annotations

import numpy as np


def tiles_touched(rect: np.ndarray, visible: np.ndarray, tile_w: int, tile_h: int) -> np.ndarray:
    n = rect.shape[0]
    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        if not visible[i]:
            continue
        x0, y0, x1, y1 = (int(v) for v in rect[i])
        out[i] = (x1 // tile_w - x0 // tile_w + 1) * (y1 // tile_h - y0 // tile_h + 1)
    return out


def bin_gaussians(rect: np.ndarray, depth: np.ndarray, visible: np.ndarray,
                  width: int, height: int, tile_w: int, tile_h: int):
    """Returns (sorted_ids uint32[M], sorted_tiles int64[M], ranges uint32[n_tiles, 2])."""
    tiles_x = (width + tile_w - 1) // tile_w
    tiles_y = (height + tile_h - 1) // tile_h
    tile_ids, depths, ids = [], [], []
    for i in np.flatnonzero(visible):
        x0, y0, x1, y1 = (int(v) for v in rect[i])
        for ty in range(y0 // tile_h, y1 // tile_h + 1):
            for tx in range(x0 // tile_w, x1 // tile_w + 1):
                tile_ids.append(ty * tiles_x + tx)
                depths.append(depth[i])
                ids.append(i)
    tile_ids = np.asarray(tile_ids, dtype=np.int64)
    depths = np.asarray(depths)
    ids = np.asarray(ids, dtype=np.int64)
    order = np.lexsort((ids, depths, tile_ids))
    st, sd = tile_ids[order], ids[order]
    n_tiles = tiles_x * tiles_y
    counts = np.bincount(st, minlength=n_tiles)
    ends = np.cumsum(counts)
    ranges = np.stack([ends - counts, ends], axis=1).astype(np.uint32)
    return sd.astype(np.uint32), st, ranges


def reached_pairs(rect, uv, conic, q, visible, width: int, tile_w: int, tile_h: int) -> np.ndarray:
    """(tile id, Gaussian index) pairs, as sorted keys tile_id * n + index, of
    the tiles holding a pixel centre inside the Gaussian's cut-level ellipse
    a dx^2 + 2 b dx dy + c dy^2 <= q, (dx, dy) = (px + 0.5 - u, py + 0.5 - v):
    the tiles in which its alpha can reach alpha_min.  Every pixel of the
    Gaussian's rectangle is tested."""
    n = rect.shape[0]
    tiles_x = (width + tile_w - 1) // tile_w
    keys = []
    for i in np.flatnonzero(visible):
        x0, y0, x1, y1 = (int(v) for v in rect[i])
        px = np.arange(x0, x1 + 1)
        py = np.arange(y0, y1 + 1)
        dx = (px + 0.5 - uv[i, 0])[None, :]
        dy = (py + 0.5 - uv[i, 1])[:, None]
        a, b, c = conic[i]
        inside = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy <= q[i]
        yy, xx = np.nonzero(inside)
        t = np.unique((py[yy] // tile_h) * tiles_x + px[xx] // tile_w)
        keys.append(t.astype(np.int64) * n + i)
    return np.sort(np.concatenate(keys)) if keys else np.zeros(0, dtype=np.int64)
