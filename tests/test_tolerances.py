"""The oracle's flag windows against the float32 exponent the compositors use,
checked on the CPU.

The image tolerance exempts a pixel only when one of its decisions sits within
the oracle's window of a threshold (alpha within rel_alpha of alpha_min).  That
is sound if a float32 evaluation of alpha stays within the window of the FP64
one.  The compositor evaluates log2(opacity G) with the square completed in y
from quantities the preprocess forms in float64 (both variable terms of one
sign) at offsets from the centre of the 32x32 pixel block; the float32 steps are
written out below in that order (a product of two float32 values is exact in
float64, so fma(a, b, c) is (a * b + c) in float64 rounded once), on a scene
full of needles centred far outside the image, where a direct float32
evaluation of -1/2 d^T conic d would lose digits to cancellation."""
import math

import numpy as np

from oracle import composite as oc
from paper_2503_16422_amd import inputs
from tests.gpu_helpers import oracle_settings

F32 = np.float32
LOG2E = 1.0 / math.log(2.0)


def _f(x):
    return np.asarray(x, dtype=np.float64).astype(F32)


def _fma(a, b, c):
    return _f(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def _needle_pairs(n_gauss=20_000, per=48, seed=9):
    sc = inputs.tiny_scene(n_gauss, seed=seed)
    sc.log_scale[3] += 3.0                      # long-lived: many near the camera at once
    cam = inputs.look_at_camera(20.0, 3.0, 96, 72)
    st = oracle_settings()
    pre = oc.prepare(sc.arrays(), cam, 0.5, st)
    rng = np.random.default_rng(1)
    g_all, px_all, py_all = [], [], []
    for g in np.flatnonzero(pre.visible):
        x0, y0, x1, y1 = pre.rect[g]
        nx, ny = x1 - x0 + 1, y1 - y0 + 1
        k = rng.choice(nx * ny, min(per, nx * ny), replace=False)
        g_all.append(np.full(k.size, g))
        px_all.append(x0 + k % nx)
        py_all.append(y0 + k // nx)
    return pre, st, np.concatenate(g_all), np.concatenate(px_all), np.concatenate(py_all)


def _float32_exponent(pre, g, px, py):
    """log2(opacity G) as the compositor forms it (completed square, block-centred offsets)."""
    c00, c01, c11 = pre.cov2d[g, 0, 0], pre.cov2d[g, 0, 1], pre.cov2d[g, 1, 1]
    det = c00 * c11 - c01 * c01
    kx, q = _f(-0.5 * LOG2E / c00), _f(np.sqrt(0.5 * LOG2E * c00 / det))
    s = -c01 / c00
    s_hi = _f(s)
    s_lo = _f(s - s_hi.astype(np.float64))
    u, v = pre.uv[g, 0], pre.uv[g, 1]
    u_hi, v_hi = _f(u), _f(v)
    u_lo, v_lo = _f(u - u_hi.astype(np.float64)), _f(v - v_hi.astype(np.float64))
    ox = ((px & ~31) + 16).astype(np.float64)
    oy = ((py & ~31) + 16).astype(np.float64)
    gx = (u_hi.astype(np.float64) - ox) + u_lo.astype(np.float64)
    gy = (v_hi.astype(np.float64) - oy) + v_lo.astype(np.float64)
    sd = s_hi.astype(np.float64) + s_lo.astype(np.float64)
    qd = q.astype(np.float64)
    s_sc = _f(qd * sd)
    c0 = _f(-qd * (gy + sd * gx))
    lo = _f(np.log2(_f(pre.opac[g]).astype(np.float64)))
    fx = _f(px - ox + 0.5)
    fy = _f(py - oy + 0.5)
    dx = _f(fx.astype(np.float64) - _f(gx).astype(np.float64))
    A = _fma(_f(kx.astype(np.float64) * dx.astype(np.float64)), dx, lo)
    t = _fma(s_sc, fx, c0)
    w = _fma(q, fy, t)
    return _fma(-w, w, A)


def test_float32_exponent_within_the_alpha_flag_window():
    pre, st, g, px, py = _needle_pairs()
    dx = px + 0.5 - pre.uv[g, 0]
    dy = py + 0.5 - pre.uv[g, 1]
    a, b, c = pre.conic[g, 0], pre.conic[g, 1], pre.conic[g, 2]
    q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    e64 = np.log2(pre.opac[g]) - 0.5 * LOG2E * q
    near = e64 > math.log2(st.alpha_min) - 2.0            # pairs whose alpha decision can matter
    e32 = _float32_exponent(pre, g[near], px[near], py[near]).astype(np.float64)
    rel = np.abs(e32 - e64[near]) * math.log(2.0)          # relative error of alpha = 2^e
    # the cancellation this scene exercises: the quadratic form's terms exceed
    # their sum by orders of magnitude at many of these pairs
    terms = np.abs(a * dx * dx) + 2 * np.abs(b * dx * dy) + np.abs(c * dy * dy)
    ratio = terms[near] / np.maximum(q[near], 1e-30)
    print(f"terms / form: max {ratio.max():.1e}, {(ratio > 1e3).sum()} pairs above 1e3")
    assert (ratio > 1e3).sum() >= 100
    window = 2e-5        # the oracle's rel_alpha
    assert near.sum() > 100_000
    assert rel.max() <= 0.75 * window, float(rel.max())
    print(f"{near.sum()} pairs near alpha_min: max relative alpha error {rel.max():.2e}, "
          f"99.99% {np.quantile(rel, 0.9999):.2e}")
