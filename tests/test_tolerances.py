"""The image tolerances the GPU parity tests use, checked on the CPU.

cancellation_bound widens the image tolerance where float32 loses digits of
the exponent to cancellation.  Here a float32 walk of the same lists (written
out below from Eq. 2 and the front-to-back blend, in the order a float32
compositor evaluates them) must stay within 1e-5 + that bound of the FP64
oracle on every unflagged pixel of a scene with near-camera needles, and the
scene must hold pixels where the plain 1e-4 tolerance would not be enough."""
import numpy as np

from oracle import binning as obin
from oracle import composite as oc
from paper_2503_16422_amd import inputs
from tests.gpu_helpers import cancellation_bound, oracle_settings


def _float32_walk(pre, ids, ranges, W, H, tw, th, st):
    f32 = np.float32
    uv, con = pre.uv.astype(f32), pre.conic.astype(f32)
    op, col = pre.opac.astype(f32), pre.rgb.astype(f32)
    amin, amax, tmin = f32(st.alpha_min), f32(st.alpha_max), f32(st.t_min)
    out = np.zeros((3, H, W))
    tx_n = (W + tw - 1) // tw
    for t in range(ranges.shape[0]):
        ty, tx = divmod(t, tx_n)
        ys, xs = np.meshgrid(np.arange(ty * th, min(H, ty * th + th)), np.arange(tx * tw, min(W, tx * tw + tw)),
                             indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
        sx, sy = xs.astype(f32) + f32(0.5), ys.astype(f32) + f32(0.5)
        T = np.ones(xs.size, f32)
        C = np.zeros((3, xs.size), f32)
        live = np.ones(xs.size, bool)
        for k in range(ranges[t, 0], ranges[t, 1]):
            if not live.any():
                break
            i = ids[k]
            dx, dy = sx - uv[i, 0], sy - uv[i, 1]
            pw = f32(-0.5) * (con[i, 0] * dx * dx + con[i, 2] * dy * dy) - con[i, 1] * dx * dy
            al = np.minimum(amax, op[i] * np.exp(pw))
            use = live & (al >= amin)
            test = T * (f32(1) - al)
            live &= ~(use & (test < tmin))
            use &= live
            C += np.where(use, col[i][:, None] * (al * T), f32(0))
            T = np.where(use, test, T)
        out[:, ys, xs] = C
    return out


def test_cancellation_bound_covers_a_float32_walk():
    sc = inputs.tiny_scene(60_000, seed=9)
    sc.log_scale[3] += 3.0
    W, H = 48, 36
    cam = inputs.look_at_camera(20.0, 3.0, W, H)
    st = oracle_settings(tile_w=16, tile_h=16)
    pre = oc.prepare(sc.arrays(), cam, 0.5, st)
    ids, _, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, W, H, 16, 16)
    ref = oc.composite(pre, cam, st, mode="rect")
    bound = cancellation_bound(pre, ids, ranges, W, H, 16, 16, st)
    err = np.abs(_float32_walk(pre, ids, ranges, W, H, 16, 16, st) - ref.rgb).max(axis=0)
    clean = ref.flags == 0
    assert np.all(err[clean] <= 1e-5 + bound[clean]), float((err - bound)[clean].max())
    assert err[clean].max() > 1e-4, "no pixel needs the bound: the scene does not exercise it"
