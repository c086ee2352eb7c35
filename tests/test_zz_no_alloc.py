"""fdgs_build_active_mask_noalloc (no device allocation, static scratch)
against fdgs_build_active_mask, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2503_16422_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _spec(frames, key_lo, key_hi, mode, views):
    ft = np.ascontiguousarray(np.asarray(frames, dtype=np.float64))
    cams = (_lib.Camera * max(len(views), 1))(*[_lib.camera_struct(v) for v in views])
    spec = _lib.MaskSpec()
    spec.frame_times = ft.ctypes.data
    spec.n_frames = ft.size
    spec.views = ctypes.cast(cams, ctypes.c_void_p)
    spec.n_views = len(views)
    spec.key_lo, spec.key_hi = float(key_lo), float(key_hi)
    spec.mode = int(mode)
    spec.alpha_min = 0.0
    spec.dilation = -1.0
    return spec, (ft, cams)


def _noalloc(model, frames, key_lo, key_hi, mode, views):
    lib = _lib.load()
    n = model.n
    bits = torch.full(((n + 31) // 32,), -1, dtype=torch.int32, device="cuda")
    idx = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    spec, keep = _spec(frames, key_lo, key_hi, mode, views)
    ms = model.struct()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.fdgs_build_active_mask_noalloc(ctypes.byref(ms), ctypes.byref(spec),
                                                  ctypes.c_void_p(bits.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                                  ctypes.c_void_p(count.data_ptr()), stream))
    del keep
    return bits, idx, count


def _same(a, b):
    bits_a, idx_a, cnt_a = a
    bits_b, idx_b, cnt_b = b
    n = int(cnt_b.item())
    assert int(cnt_a.item()) == n
    assert torch.equal(bits_a, bits_b)
    assert torch.equal(idx_a[:n], idx_b[:n])
    return n


@pytest.mark.parametrize("mode", [_lib.MASK_TEMPORAL, _lib.MASK_TEMPORAL_AND_TILE])
def test_noalloc_mask_matches_allocating_entry_point_twice(mode):
    from paper_2503_16422_amd.render import Context, GaussianModel
    ctx = Context(0)
    views = inputs.arc_cameras(5, 4.0, 338, 254)
    frames = inputs.frame_times(300)
    # a large call, then a smaller one: the shared scratch keeps the first call's contents
    for n, seed, lo, hi in ((150_000, 3, 110, 120), (7_001, 4, 200, 210)):
        sc = inputs.long_scene(n, seed=seed)
        model = GaussianModel.from_scene(sc, "cuda:0")
        win = frames[lo:hi + 1]
        ref = ctx.build_active_mask(model, win, frames[lo], frames[hi], mode, views)
        got = _noalloc(model, win, frames[lo], frames[hi], mode, views)
        torch.cuda.synchronize()
        kept = _same(got, ref)
        assert 0 < kept < n
    ctx.close()


def test_noalloc_mask_rejects_what_it_cannot_do():
    from paper_2503_16422_amd.render import GaussianModel
    lib = _lib.load()
    sc = inputs.long_scene(1000, seed=1)
    model = GaussianModel.from_scene(sc, "cuda:0")
    views = inputs.arc_cameras(2, 4.0, 64, 48)
    spec, keep = _spec([], 0.3, 0.4, _lib.MASK_CONTRIBUTED, views)
    ms = model.struct()
    buf = torch.zeros(2048, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert lib.fdgs_build_active_mask_noalloc(ctypes.byref(ms), ctypes.byref(spec), p, p, p,
                                              None) == _lib.FDGS_ERR_UNSUPPORTED
    spec, keep2 = _spec([0.3, 0.35], 0.3, 0.35, _lib.MASK_TEMPORAL, [])
    big = model.struct()
    big.n = (1 << 27) + 1        # rejected on the host before any device access
    assert lib.fdgs_build_active_mask_noalloc(ctypes.byref(big), ctypes.byref(spec), p, p, p,
                                              None) == _lib.FDGS_ERR_INVALID_ARG
    assert b"exceeds" in lib.fdgs_last_error()
