"""Keyframe active sets (Sec. 4.2.2), FP64 (test infrastructure only).

Keyframes sit at even intervals; a frame is rendered with the union of the
active sets of its two nearest keyframes.  The paper builds each keyframe's
set from training-view visibility; the predicates computed here are:

  TEMPORAL (mode 0): keep Gaussian i iff its temporal opacity p_i(t) (Eq. 3)
      reaches 1/255 at some frame of the window, i.e.
          min_f (t_f - mu_t)^2 <= 2 ln(255) Sigma_44.
      A Gaussian outside this set has sigma_i p_i(t) < 1/255 at every frame of
      the window, so it never passes the alpha test: masked and unmasked
      renders of the window are identical.

  TEMPORAL_AND_TILE (mode 1): additionally require that, at one of the two
      keyframe times, the Gaussian's opacity-free footprint (the rectangle at
      Mahalanobis level 2 ln 255, as in `composite.pixel_rects` with culling
      off) covers at least one pixel of at least one mask view.

  CONTRIBUTED (mode 2): the paper's keyframe visibility: keep Gaussian i iff
      it is blended (Eq. 2: alpha >= alpha_min and the pixel's walk has not
      stopped) at some pixel of some mask view rendered at key_lo or at
      key_hi; the window's set is the union over views and both keyframes.
      The window's frame times are not used.  Rendering a keyframe from a
      mask view with this set gives exactly the unmasked image.

Output: LSB-first bit words and the ascending kept indices.
"""
from __future__ import annotations

import math

import numpy as np

from .composite import Settings, composite, pixel_rects, prepare
from .projection import project
from .slicing import covariance_4d, rows, slice_at, valid_gaussians

TEMPORAL = 0
TEMPORAL_AND_TILE = 1
CONTRIBUTED = 2


def temporal_keep(mean_t: np.ndarray, sigma44: np.ndarray, frame_times, alpha_min=1.0 / 255.0):
    level = 2.0 * math.log(1.0 / alpha_min)
    keep = np.zeros(mean_t.shape, dtype=bool)
    for tf in frame_times:
        d = float(tf) - mean_t
        keep |= d * d <= level * sigma44
    return keep


def spatial_keep(scene_arrays, views, key_times, dilation: float = 0.3,
                 alpha_min: float = 1.0 / 255.0):
    mean, log_scale, q_l, q_r, logit = scene_arrays[:5]
    M, LS, QL, QR = rows(mean), rows(log_scale), rows(q_l), rows(q_r)
    valid = valid_gaussians(M, LS, QL, QR, np.asarray(logit, dtype=np.float64))
    M, LS = np.where(valid[:, None], M, 0.0), np.where(valid[:, None], LS, 0.0)
    QL, QR = np.where(valid[:, None], QL, 1.0), np.where(valid[:, None], QR, 1.0)
    st = Settings(alpha_min=alpha_min, dilation=dilation, temporal_cull=False)
    keep = np.zeros(M.shape[0], dtype=bool)
    for tk in key_times:
        mean3, cov3, _ = slice_at(M, LS, QL, QR, float(tk))
        for cam in views:
            uv, cov2d, _, ok = project(mean3, cov3, cam, dilation)
            r = pixel_rects(uv, cov2d, np.ones(M.shape[0]), cam.width, cam.height, st)
            keep |= ok & (r[:, 0] <= r[:, 2]) & (r[:, 1] <= r[:, 3])
    return keep & valid


def contributed_keep(scene_arrays, views, key_times, st: Settings):
    """(sure, maybe) bool[n]: blended at some pixel of some view at some key
    time, with every decision on the way clear of the thresholds (sure), or
    blended or possibly blended by a float32 walk (maybe)."""
    n = scene_arrays[0].shape[1]
    sure = np.zeros(n, dtype=bool)
    maybe = np.zeros(n, dtype=bool)
    for tk in key_times:
        for cam in views:
            pre = prepare(scene_arrays, cam, float(tk), st)
            c = composite(pre, cam, st, mode="rect", contributions=True).contrib
            sure |= (c & 1) != 0
            maybe |= (c & 2) != 0
    return sure, maybe


def active_mask(scene_arrays, frame_times, key_lo: float, key_hi: float, mode: int = TEMPORAL,
                views=(), dilation: float = 0.3, alpha_min: float = 1.0 / 255.0):
    """Returns (keep bool[n], bits uint32[ceil(n/32)], idx uint32[count])."""
    mean, log_scale, q_l, q_r, logit = scene_arrays[:5]
    M, LS, QL, QR = rows(mean), rows(log_scale), rows(q_l), rows(q_r)
    valid = valid_gaussians(M, LS, QL, QR, np.asarray(logit, dtype=np.float64))
    LS_ = np.where(valid[:, None], LS, 0.0)
    QL_, QR_ = np.where(valid[:, None], QL, 1.0), np.where(valid[:, None], QR, 1.0)
    sigma44 = covariance_4d(LS_, QL_, QR_)[:, 3, 3]
    keep = valid & temporal_keep(np.where(valid, M[:, 3], 0.0), sigma44, frame_times, alpha_min)
    if mode == TEMPORAL_AND_TILE:
        keep &= spatial_keep(scene_arrays, views, (key_lo, key_hi), dilation, alpha_min)
    elif mode != TEMPORAL:
        raise ValueError(mode)
    return keep, pack_bits(keep), np.flatnonzero(keep).astype(np.uint32)


def pack_bits(keep: np.ndarray) -> np.ndarray:
    """Bit i of word i // 32 (LSB first) is keep[i]."""
    n = keep.shape[0]
    nw = (n + 31) // 32
    padded = np.zeros(nw * 32, dtype=np.uint64)
    padded[:n] = keep
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    return (padded.reshape(nw, 32) * weights).sum(axis=1).astype(np.uint32)
