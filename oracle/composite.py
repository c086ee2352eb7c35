"""Per-pixel front-to-back compositing, FP64 (test infrastructure only).

Eq. 2: I(u, v, t) = sum_i c_i(d) alpha_i prod_{j<i} (1 - alpha_j) over the
Gaussians sorted by depth; Eq. 3: alpha_i = p_i(t) * G_2D(u, v) * sigma_i.

Readings where the paper is silent (the usual 3D Gaussian Splatting rules):
  * alpha is clamped to alpha_max = 0.99, an alpha below alpha_min = 1/255 is
    skipped, and the walk stops before a Gaussian that would take the
    transmittance below t_min = 1e-4;
  * depth = camera-space z of the conditional mean; equal depths are ordered
    by the Gaussian's index;
  * the background is added with the final transmittance.

Two walks: `composite_py` (pure Python, for a handful of Gaussians and
pixels) and `composite` (the same walk in C with OpenMP).  Rect mode skips a
Gaussian at pixels outside its conservative pixel rectangle (see
`pixel_rects`), where alpha < alpha_min is certain.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np

from . import build as _build
from .projection import camera_center, project
from .sh import sh_color
from .slicing import rows, sigmoid, slice_at, valid_gaussians

RECT_MARGIN_REL = 1e-4
RECT_MARGIN_ABS = 1e-4


@dataclasses.dataclass
class Settings:
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    dilation: float = 0.3
    bg: tuple = (0.0, 0.0, 0.0)
    temporal_cull: bool = True
    tile_w: int = 16
    tile_h: int = 16


@dataclasses.dataclass
class Prepared:
    """Per processed Gaussian quantities, FP64, in processing order."""
    alive: np.ndarray       # bool: valid, in front of znear, det > 0
    mean3: np.ndarray
    cov3: np.ndarray
    p: np.ndarray
    sigma: np.ndarray
    opac: np.ndarray        # sigma * p
    uv: np.ndarray
    cov2d: np.ndarray
    conic: np.ndarray       # (n, 3): a, b, c of Sigma_2D^{-1}
    depth: np.ndarray
    rgb: np.ndarray
    rect: np.ndarray        # (n, 4) int32 inclusive pixel rect, x0 > x1 when empty
    visible: np.ndarray     # alive and non-empty rect (and opac >= alpha_min when culling)


def prepare(scene_arrays, cam, t: float, st: Settings, idx=None) -> Prepared:
    """Slice, project and shade every Gaussian (or those in idx, in that order)."""
    mean, log_scale, q_l, q_r, logit, sh = scene_arrays[:6]
    degree = scene_arrays[6] if len(scene_arrays) > 6 else 3
    if idx is not None:
        idx = np.asarray(idx, dtype=np.int64)
        mean, log_scale, q_l, q_r = mean[:, idx], log_scale[:, idx], q_l[:, idx], q_r[:, idx]
        logit, sh = logit[idx], sh[:, :, idx]
    M, LS, QL, QR = rows(mean), rows(log_scale), rows(q_l), rows(q_r)
    lg = np.asarray(logit, dtype=np.float64)
    n = M.shape[0]
    valid = valid_gaussians(M, LS, QL, QR, lg)
    safe = lambda a, fill: np.where(valid[:, None], a, fill)
    M_, LS_ = safe(M, 0.0), safe(LS, 0.0)
    QL_, QR_ = safe(QL, 1.0), safe(QR, 1.0)
    mean3, cov3, p = slice_at(M_, LS_, QL_, QR_, t)
    sigma = sigmoid(np.where(valid, lg, 0.0))
    opac = sigma * p
    uv, cov2d, depth, ok = project(mean3, cov3, cam, st.dilation)
    alive = valid & ok
    det = cov2d[:, 0, 0] * cov2d[:, 1, 1] - cov2d[:, 0, 1] ** 2
    det = np.where(alive, det, 1.0)
    conic = np.stack([cov2d[:, 1, 1] / det, -cov2d[:, 0, 1] / det, cov2d[:, 0, 0] / det], axis=1)
    C = camera_center(cam)
    dvec = mean3 - C
    dvec /= np.linalg.norm(dvec, axis=1, keepdims=True)
    sh_rows = np.transpose(np.asarray(sh, dtype=np.float64), (2, 0, 1))
    rgb = sh_color(sh_rows, dvec, degree)
    rect = pixel_rects(uv, cov2d, opac, cam.width, cam.height, st)
    nonempty = (rect[:, 0] <= rect[:, 2]) & (rect[:, 1] <= rect[:, 3])
    visible = alive & nonempty
    if st.temporal_cull:
        visible &= opac >= st.alpha_min
    return Prepared(alive, mean3, cov3, p, sigma, opac, uv, cov2d, conic, depth, rgb, rect, visible)


def cut_level(opac: np.ndarray, st: Settings) -> np.ndarray:
    """Mahalanobis level q beyond which alpha < alpha_min, with a safety margin.

    alpha = opac * exp(-q/2) >= alpha_min  <=>  q <= 2 ln(opac / alpha_min).
    Without temporal culling the level ignores the opacity (q = 2 ln(1/alpha_min)),
    which is what a renderer that bins every Gaussian does.
    """
    if st.temporal_cull:
        ratio = np.maximum(opac / st.alpha_min, 1.0)
        q = 2.0 * np.log(ratio)
    else:
        q = np.full(opac.shape, 2.0 * math.log(1.0 / st.alpha_min))
    return q * (1.0 + RECT_MARGIN_REL) + RECT_MARGIN_ABS


def pixel_rects(uv, cov2d, opac, width, height, st: Settings) -> np.ndarray:
    """Inclusive pixel rectangle of pixel centres inside the ellipse's bounding box.

    The ellipse {d : d^T Sigma_2D^{-1} d <= q} has half-extents sqrt(q Sxx),
    sqrt(q Syy); pixel px is inside iff |px + 0.5 - u| <= hx.
    """
    q = cut_level(opac, st)
    hx = np.sqrt(q * np.maximum(cov2d[:, 0, 0], 0.0))
    hy = np.sqrt(q * np.maximum(cov2d[:, 1, 1], 0.0))
    big = 1e9
    clip = lambda a, hi: np.clip(np.nan_to_num(a, nan=-big, posinf=big, neginf=-big), -1.0, hi + 1.0)
    x0 = np.ceil(clip(uv[:, 0] - hx - 0.5, width))
    x1 = np.floor(clip(uv[:, 0] + hx - 0.5, width))
    y0 = np.ceil(clip(uv[:, 1] - hy - 0.5, height))
    y1 = np.floor(clip(uv[:, 1] + hy - 0.5, height))
    x0, y0 = np.maximum(x0, 0), np.maximum(y0, 0)
    x1, y1 = np.minimum(x1, width - 1), np.minimum(y1, height - 1)
    return np.stack([x0, y0, x1, y1], axis=1).astype(np.int32)


def depth_order(pre: Prepared, use_visible: bool = False) -> np.ndarray:
    """Indices of the alive (or visible) Gaussians sorted by (depth, index)."""
    keep = pre.visible if use_visible else pre.alive
    ids = np.flatnonzero(keep)
    return ids[np.lexsort((ids, pre.depth[ids]))]


def composite_py(pre: Prepared, order, px, py, st: Settings):
    """The per-pixel walk, written as plain Python loops.  Returns rgb (3,), T."""
    sx, sy = px + 0.5, py + 0.5
    T, C = 1.0, np.zeros(3)
    for i in order:
        dx, dy = sx - pre.uv[i, 0], sy - pre.uv[i, 1]
        a, b, c = pre.conic[i]
        power = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy)
        alpha = min(st.alpha_max, pre.opac[i] * math.exp(power))
        if alpha < st.alpha_min:
            continue
        test = T * (1.0 - alpha)
        if test < st.t_min:
            break
        C = C + pre.rgb[i] * (alpha * T)
        T = test
    return C + T * np.asarray(st.bg, dtype=np.float64), T


class _Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                ("u", "v", "ca", "cb", "cc", "opac", "rgb", "depth", "rect", "contrib", "weight",
                 "weight_slack")] + [
                ("bg", ctypes.c_double * 3), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double),
                ("rel_alpha", ctypes.c_double), ("rel_t", ctypes.c_double),
                ("rel_depth", ctypes.c_double)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _LIB = ctypes.CDLL(path)
        _LIB.oracle_composite.restype = ctypes.c_int
        _LIB.oracle_num_threads.restype = ctypes.c_int
    return _LIB


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


@dataclasses.dataclass
class Image:
    rgb: np.ndarray     # (3, npix) or (3, H, W)
    T: np.ndarray
    flags: np.ndarray
    contrib: np.ndarray = None   # int32 per processed Gaussian: 1 surely blended, 2 possibly blended
    weight: np.ndarray = None    # float64 per processed Gaussian: summed alpha T over the pixels
    weight_slack: np.ndarray = None   # float64 per processed Gaussian: weight a float32 walk may move at flagged pixels


def composite(pre: Prepared, cam, st: Settings, *, mode: str = "rect", pixels=None,
              rel_alpha: float = 2e-5, rel_t: float = 1e-4, rel_depth: float = 1e-12,
              contributions: bool = False, weights: bool = False) -> Image:
    """Shade the full image (pixels=None) or the given (px, py) arrays.

    mode "brute": every alive Gaussian at every pixel; "rect": skip outside the
    conservative rectangle (identical result).  contributions: also return,
    per processed Gaussian, whether some pixel blends it (Eq. 2): bit 1 when a
    pixel does so with every decision so far clear of the thresholds, bit 2
    when a pixel does or, at a flagged pixel, may.  weights: also return, per
    processed Gaussian, the sum over the shaded pixels of its blend weight
    alpha_i T_i (the summand of Eq. 4), and in `weight_slack` the most a
    float32 walk can move that sum at the flagged pixels (see the C source).
    """
    order = depth_order(pre, use_visible=False)
    keep = np.ones(order.shape, dtype=bool)
    if mode == "rect":
        r = pre.rect[order]
        keep = (r[:, 0] <= r[:, 2]) & (r[:, 1] <= r[:, 3]) & (pre.opac[order] >= st.alpha_min)
    elif mode != "brute":
        raise ValueError(mode)
    order = order[keep]
    c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    u, v = c(pre.uv[order, 0]), c(pre.uv[order, 1])
    ca, cb, cc = c(pre.conic[order, 0]), c(pre.conic[order, 1]), c(pre.conic[order, 2])
    opac, rgb, depth = c(pre.opac[order]), c(pre.rgb[order]), c(pre.depth[order])
    rect = np.ascontiguousarray(pre.rect[order], dtype=np.int32) if mode == "rect" else None
    if pixels is None:
        py, px = np.meshgrid(np.arange(cam.height, dtype=np.int32),
                             np.arange(cam.width, dtype=np.int32), indexing="ij")
        px, py = px.ravel(), py.ravel()
        full = True
    else:
        px = np.asarray(pixels[0], dtype=np.int32)
        py = np.asarray(pixels[1], dtype=np.int32)
        full = False
    perm = np.lexsort((px, py))
    spx, spy = np.ascontiguousarray(px[perm]), np.ascontiguousarray(py[perm])
    npix = spx.shape[0]
    out_rgb = np.zeros((npix, 3))
    out_t = np.zeros(npix)
    out_f = np.zeros(npix, dtype=np.int32)
    s = _Scene()
    s.n = order.shape[0]
    ptr = lambda a: a.ctypes.data if a is not None else None
    s.u, s.v, s.ca, s.cb, s.cc = ptr(u), ptr(v), ptr(ca), ptr(cb), ptr(cc)
    s.opac, s.rgb, s.depth, s.rect = ptr(opac), ptr(rgb), ptr(depth), ptr(rect)
    contrib = np.zeros(order.shape[0], dtype=np.int32) if contributions else None
    s.contrib = ptr(contrib)
    weight = np.zeros(order.shape[0]) if weights else None
    s.weight = ptr(weight)
    slack = np.zeros(order.shape[0]) if weights else None
    s.weight_slack = ptr(slack)
    for k in range(3):
        s.bg[k] = float(st.bg[k])
    s.alpha_min, s.alpha_max, s.t_min = st.alpha_min, st.alpha_max, st.t_min
    s.rel_alpha, s.rel_t, s.rel_depth = rel_alpha, rel_t, rel_depth
    rc = _lib().oracle_composite(ctypes.byref(s), ctypes.c_int64(npix),
                                 spx.ctypes.data_as(ctypes.c_void_p), spy.ctypes.data_as(ctypes.c_void_p),
                                 out_rgb.ctypes.data_as(ctypes.c_void_p),
                                 out_t.ctypes.data_as(ctypes.c_void_p),
                                 out_f.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise MemoryError("oracle_composite failed")
    inv = np.empty_like(perm)
    inv[perm] = np.arange(npix)
    rgb_o, t_o, f_o = out_rgb[inv].T, out_t[inv], out_f[inv]
    per_gauss = per_w = per_s = None
    if contributions:
        per_gauss = np.zeros(pre.visible.shape[0], dtype=np.int32)
        per_gauss[order] = contrib
    if weights:
        per_w = np.zeros(pre.visible.shape[0])
        per_w[order] = weight
        per_s = np.zeros(pre.visible.shape[0])
        per_s[order] = slack
    if full:
        H, W = cam.height, cam.width
        return Image(rgb_o.reshape(3, H, W), t_o.reshape(H, W), f_o.reshape(H, W), per_gauss, per_w, per_s)
    return Image(rgb_o, t_o, f_o, per_gauss, per_w, per_s)


def render(scene_arrays, cam, t: float, st: Settings = None, *, idx=None, mode="rect",
           pixels=None, **flag_kw) -> Image:
    st = st or Settings()
    pre = prepare(scene_arrays, cam, t, st, idx=idx)
    return composite(pre, cam, st, mode=mode, pixels=pixels, **flag_kw)
