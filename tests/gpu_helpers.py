"""Shared helpers for the GPU parity tests (inputs and tolerances only)."""
import numpy as np
import pytest

from oracle import composite as oc

F32 = lambda x: float(np.float32(x))

# Image tolerance: max |GPU - FP64 oracle| per channel, over pixels the oracle
# does not flag as sitting within 1e-5 (alpha) / 1e-4 (transmittance) of a
# threshold decision.
IMG_TOL = 1e-4
# A flagged pixel can differ by at most one near-threshold contribution.
FLAG_TOL = 2e-2
# Expected flagged fraction: ~(pairs evaluated per pixel) x (2e-5 / ln(255)),
# e.g. 225 pairs/pixel at 1352x1014 -> ~0.08%.  Allow a few times that.
MAX_FLAGGED_FRAC = 5e-3


def oracle_settings(cfg=None, **kw) -> oc.Settings:
    """Oracle settings with the float32 values the library receives."""
    base = dict(alpha_min=F32(1 / 255), alpha_max=F32(0.99), t_min=F32(1e-4), dilation=F32(0.3),
                bg=(0.0, 0.0, 0.0), temporal_cull=True, tile_w=16, tile_h=16)
    if cfg is not None:
        base.update(alpha_min=float(cfg.alpha_min), alpha_max=float(cfg.alpha_max), t_min=float(cfg.t_min),
                    dilation=float(cfg.dilation), bg=tuple(float(cfg.bg[i]) for i in range(3)),
                    temporal_cull=bool(cfg.temporal_cull), tile_w=cfg.tile_w, tile_h=cfg.tile_h)
    base.update(kw)
    return oc.Settings(**base)


def compare_image(gpu_rgb, ref, *, tol=IMG_TOL, pixels=None, extra=None, max_flagged=MAX_FLAGGED_FRAC):
    """gpu_rgb (3, H, W) numpy; ref an oracle Image (full or sampled).
    extra: per-pixel allowance added to both tolerances (cancellation_bound);
    max_flagged: allowed fraction of flagged pixels."""
    if pixels is None:
        g = gpu_rgb.reshape(3, -1)
        r = ref.rgb.reshape(3, -1)
        f = ref.flags.reshape(-1)
    else:
        px, py = pixels
        g = gpu_rgb[:, py, px]
        r = ref.rgb
        f = ref.flags
    err = np.abs(g - r).max(axis=0)
    if extra is not None:
        err = np.maximum(err - np.asarray(extra).reshape(-1), 0.0)
    clean = f == 0
    n_flag = int((~clean).sum())
    worst = float(err[clean].max()) if clean.any() else 0.0
    worst_flag = float(err[~clean].max()) if n_flag else 0.0
    assert worst <= tol, f"max |err| {worst:.3e} over unflagged pixels"
    assert n_flag <= max(2, max_flagged * f.size), f"{n_flag} flagged pixels"
    assert worst_flag <= FLAG_TOL, f"flagged pixel error {worst_flag:.3e}"
    return worst, n_flag


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check_culled_binning(b, pre, st, W, H, tile_w, tile_h):
    """Tile lists of a forward with tile culling, against the oracle's binning.

    Each tile's list must be the oracle's rectangle list (depth order) with
    some Gaussians left out, and must keep every Gaussian whose cut-level
    ellipse holds a pixel centre of the tile.  Returns (GPU instances,
    rectangle instances, reached pairs)."""
    from oracle import binning as obin
    n = pre.rect.shape[0]
    ids_a, tiles_a, _ = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, W, H, tile_w, tile_h)
    key_a = tiles_a.astype(np.int64) * n + ids_a.astype(np.int64)      # rectangle lists, in list order
    ranges = b["tile_ranges"].cpu().numpy().astype(np.int64)
    ids_g = b["sorted_ids"].cpu().numpy().astype(np.int64)
    tile_g = np.zeros(ids_g.size, dtype=np.int64)
    for t in np.flatnonzero(ranges[:, 1] > ranges[:, 0]):
        tile_g[ranges[t, 0]:ranges[t, 1]] = t
    assert np.all(np.diff(ranges[:, 0]) >= 0) and ranges[-1, 1] <= ids_g.size
    key_g = tile_g * n + ids_g
    # positions of the GPU pairs in the rectangle lists: present and increasing
    order = np.argsort(key_a, kind="stable")
    at = np.searchsorted(key_a[order], key_g)
    at = np.minimum(at, key_a.size - 1)
    assert np.all(key_a[order][at] == key_g), "a listed pair outside the Gaussian's rectangle"
    pos = order[at]
    assert np.all(np.diff(pos) > 0), "a tile list is out of depth order"
    q = oc.cut_level(pre.opac, st)
    need = obin.reached_pairs(pre.rect, pre.uv, pre.conic, q, pre.visible, W, tile_w, tile_h)
    missing = np.setdiff1d(need, key_g)
    assert missing.size == 0, f"{missing.size} reached (tile, Gaussian) pairs dropped, first {missing[:4]}"
    return ids_g.size, ids_a.size, need.size


def cancellation_bound(pre, ids, ranges, W, H, tile_w, tile_h, st, pixels=None, chunk=512, walked=False):
    """Per-pixel bound (3-channel max) on how far a float32 compositor may sit
    from the FP64 image because of cancellation in the exponent.

    The exponent -q/2 with q = a dx^2 + 2 b dx dy + c dy^2 (Eq. 2's Gaussian
    at the pixel) is summed from terms whose magnitudes add up to
    Q = |a| dx^2 + 2 |b dx dy| + |c| dy^2.  Far from a needle-shaped
    Gaussian's centre Q can exceed q by four orders of magnitude, and float32
    rounding of the terms (and of dx, dy) moves the exponent by up to about
    4 eps32 Q, so alpha by that relative amount.  The colour's derivative in
    alpha_i is bounded by 2 T_i max|c| (the Gaussian's own term plus the
    change of every later transmittance), which gives, to first order,
        |dC| <= sum_i 2 max|c| T_i alpha_i 4 eps32 Q_i
    over the blended Gaussians of the pixel, walked in the oracle's FP64 list
    order with its thresholds.  ids / ranges are the oracle's tile lists.
    Returns (H, W), or one value per (px, py) pixel when `pixels` is given;
    with walked=True also the mean number of list entries a pixel evaluates."""
    eps = float(np.finfo(np.float32).eps)
    cmax = float(np.abs(pre.rgb).max()) if pre.rgb.size else 0.0
    if pixels is None:
        yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        px, py = xx.ravel(), yy.ravel()
    else:
        px, py = (np.asarray(v, dtype=np.int64) for v in pixels)
    tile = (py // tile_h) * ((W + tile_w - 1) // tile_w) + px // tile_w
    out = np.zeros(px.size)
    n_walked = 0
    for t in np.unique(tile):
        sel = np.flatnonzero(tile == t)
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        sx, sy = px[sel] + 0.5, py[sel] + 0.5
        T = np.ones(sel.size)
        acc = np.zeros(sel.size)
        live = np.ones(sel.size, bool)
        for k0 in range(s, e, chunk):
            if not live.any():
                break
            g = ids[k0:min(k0 + chunk, e)].astype(np.int64)
            dx = sx[None, :] - pre.uv[g, 0][:, None]
            dy = sy[None, :] - pre.uv[g, 1][:, None]
            a, b, c = (pre.conic[g, j][:, None] for j in range(3))
            q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
            Q = np.abs(a) * dx * dx + 2.0 * np.abs(b * dx * dy) + np.abs(c) * dy * dy
            al = np.minimum(st.alpha_max, pre.opac[g][:, None] * np.exp(-0.5 * q))
            use = al >= st.alpha_min
            f = np.where(use, 1.0 - al, 1.0)
            after = T[None, :] * np.cumprod(f, axis=0)          # transmittance after each row
            before = after / f
            stop = use & (after < st.t_min)                      # the walk ends at the first such row
            first = np.where(stop.any(axis=0), stop.argmax(axis=0), g.size)
            blend = use & (np.arange(g.size)[:, None] < first[None, :]) & live[None, :]
            acc += (blend * before * al * Q).sum(axis=0)
            n_walked += int(np.minimum(first + 1, g.size)[live].sum())
            T = after[-1]
            live &= first == g.size
        out[sel] = 8.0 * eps * cmax * acc
    out = out.reshape(H, W) if pixels is None else out
    return (out, n_walked / max(px.size, 1)) if walked else out
