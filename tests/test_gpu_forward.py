"""GPU parity of the forward path against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from oracle import binning as obin
from oracle import composite as oc
from oracle import mask as omask
from oracle import slicing as osl
from paper_2503_16422_amd import _lib, inputs
from tests.gpu_helpers import MAX_FLAGGED_FRAC, check_culled_binning, compare_image, oracle_settings

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_16422_amd.render import Context
    c = Context(0)
    yield c
    c.close()


def to_dev(scene):
    from paper_2503_16422_amd.render import GaussianModel
    return GaussianModel.from_scene(scene, "cuda:0")


# a1/a2 ------------------------------------------------------------------------
@pytest.mark.parametrize("use_idx", [False, True])
def test_slice_4d_matches_eq1(ctx, use_idx):
    sc = inputs.tiny_scene(10_000, seed=0)
    model = to_dev(sc)
    idx = None
    sel = np.arange(sc.n)
    if use_idx:
        sel = np.sort(np.random.default_rng(1).choice(sc.n, 3001, replace=False))
        idx = torch.from_numpy(sel.astype(np.int32)).cuda()
    mean3, cov3, p = ctx.slice_4d(model, 0.5, idx)
    torch.cuda.synchronize()
    M, LS, QL, QR = (osl.rows(a)[sel] for a in (sc.mean, sc.log_scale, sc.q_left, sc.q_right))
    m_ref, c_ref, p_ref = osl.slice_at(M, LS, QL, QR, 0.5)
    g_m = mean3.cpu().numpy().T
    g_c = cov3.cpu().numpy().T
    g_p = p.cpu().numpy()
    assert np.abs(g_m - m_ref).max() <= 1e-6 * (1 + np.abs(m_ref).max())
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    c_ref6 = np.stack([c_ref[:, i, j] for i, j in iu], 1)
    scale = np.abs(c_ref6).max(axis=1, keepdims=True)
    assert (np.abs(g_c - c_ref6) <= 1e-6 * scale + 1e-30).all()
    assert np.abs(g_p - p_ref).max() <= 1e-7


# a6 image parity ------------------------------------------------------------------
def test_tiny_render_matches_oracle(ctx):
    sc = inputs.tiny_scene(10_000, seed=0)
    cam = inputs.look_at_camera(0.0, 3.0, 256, 256)
    model = to_dev(sc)
    rgb, T, _ = ctx.render(model, cam, 0.5, want_T=True)
    torch.cuda.synchronize()
    st = oracle_settings()
    ref = oc.render(sc.arrays(), cam, 0.5, st, mode="rect")
    worst, nflag = compare_image(rgb.cpu().numpy(), ref)
    assert np.abs(T.cpu().numpy() - ref.T)[ref.flags == 0].max() <= 1e-4
    print(f"tiny render: max err {worst:.2e}, flagged {nflag}")


@pytest.mark.parametrize("W,H,bg", [(37, 29, (0.0, 0.0, 0.0)), (100, 61, (0.2, 0.5, 1.0)), (1, 1, (0.3, 0.3, 0.3))])
def test_ragged_images_and_background(ctx, W, H, bg):
    sc = inputs.tiny_scene(3000, seed=4)
    sc.log_scale[:3] += 1.0
    cam = inputs.look_at_camera(10.0, 3.0, W, H)
    model = to_dev(sc)
    cfg = _lib.default_cfg(bg=bg)
    rgb, _, _ = ctx.render(model, cam, 0.4, cfg)
    torch.cuda.synchronize()
    ref = oc.render(sc.arrays(), cam, 0.4, oracle_settings(cfg), mode="brute")
    compare_image(rgb.cpu().numpy(), ref)


def test_empty_and_invisible_scenes(ctx):
    cam = inputs.look_at_camera(0.0, 3.0, 48, 40)
    cfg = _lib.default_cfg(bg=(0.25, 0.5, 0.75))
    bg = torch.tensor([0.25, 0.5, 0.75], device="cuda")[:, None, None].expand(3, 40, 48)
    rgb, T, _ = ctx.render(_empty_model(), cam, 0.5, cfg, want_T=True)
    torch.cuda.synchronize()
    assert torch.equal(rgb, bg) and torch.all(T == 1)
    # every Gaussian behind the camera
    sc = inputs.tiny_scene(500, seed=1)
    rgb, _, st = ctx.render(to_dev(sc), _looking_away(48, 40), 0.5, cfg, keep_state=True)
    b = ctx.binning(st)
    assert b["n_inst"] == 0 and b["n_vis"] == 0
    assert torch.equal(rgb, bg)
    ctx.release(st)


def _looking_away(W, H):
    c = inputs.look_at_camera(180.0, 3.0, W, H)      # at (0, 0, -3) facing the origin
    c.R = np.stack([-c.R[0], c.R[1], -c.R[2]])       # turn around, keep a right-handed frame
    c.tvec = -c.R @ np.array([0.0, 0.0, -3.0])
    return c


def _empty_model():
    from paper_2503_16422_amd.render import GaussianModel
    z = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    return GaussianModel(z(4, 0), z(4, 0), z(4, 0), z(4, 0), z(0), z(16, 3, 0))


def test_degenerate_gaussians_are_culled(ctx):
    sc = inputs.tiny_scene(400, seed=2)
    sc.log_scale[:3] += 1.0
    sc.q_left[:, 3] = 0.0          # zero quaternion
    sc.mean[0, 5] = np.nan
    sc.log_scale[1, 7] = np.inf
    sc.opacity_logit[9] = -np.inf
    cam = inputs.look_at_camera(0.0, 3.0, 64, 64)
    rgb, _, _ = ctx.render(to_dev(sc), cam, 0.5)
    torch.cuda.synchronize()
    assert torch.isfinite(rgb).all()
    keep = np.setdiff1d(np.arange(sc.n), [3, 5, 7, 9])
    ref = oc.render(sc.subset(keep).arrays(), cam, 0.5, oracle_settings(), mode="brute")
    compare_image(rgb.cpu().numpy(), ref)


# a4/a5 binning -------------------------------------------------------------------
@pytest.mark.parametrize("cull", [1, 0])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8), (32, 16), (32, 32)])
def test_binning_bit_exact(ctx, cull, tile):
    """Without tile culling the lists are exactly the rectangle binning."""
    sc = inputs.tiny_scene(10_000, seed=0)
    cam = inputs.look_at_camera(0.0, 3.0, 256, 256)
    cfg = _lib.default_cfg(temporal_cull=cull, tile_w=tile[0], tile_h=tile[1], tile_cull=0)
    rgb, _, st = ctx.render(to_dev(sc), cam, 0.5, cfg, keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    ost = oracle_settings(cfg)
    pre = oc.prepare(sc.arrays(), cam, 0.5, ost)
    vis = b["visible"].cpu().numpy().astype(bool)
    assert np.array_equal(vis, pre.visible)
    rects = b["rects"].cpu().numpy()
    assert np.array_equal(rects[vis], pre.rect[vis])
    ids, tiles, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, 256, 256, *tile)
    assert b["n_inst"] == ids.size
    assert np.array_equal(b["sorted_ids"].cpu().numpy().astype(np.uint32), ids)
    assert_same_ranges(b["tile_ranges"].cpu().numpy().astype(np.uint32), ranges)
    # and the same integer work from the library's own exported rects / depths
    ids2, _, ranges2 = obin.bin_gaussians(rects, b["depth"].cpu().numpy(), vis, 256, 256, *tile)
    assert np.array_equal(ids2, ids) and np.array_equal(ranges2, ranges)
    ctx.release(st)


@pytest.mark.parametrize("cull", [1, 0])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8), (32, 16), (32, 32)])
def test_culled_binning_between_reached_and_rectangle(ctx, cull, tile):
    """With tile culling each list is the rectangle list minus Gaussians
    whose ellipse misses the tile, in the same order, and the image is the
    unculled one bit for bit."""
    sc = inputs.tiny_scene(10_000, seed=0)
    sc.log_scale[0] += 1.5                 # elongated footprints: most of a rectangle is missed
    cam = inputs.look_at_camera(0.0, 3.0, 256, 256)
    cfg = _lib.default_cfg(temporal_cull=cull, tile_w=tile[0], tile_h=tile[1])
    model = to_dev(sc)
    rgb, _, st = ctx.render(model, cam, 0.5, cfg, keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    ost = oracle_settings(cfg)
    pre = oc.prepare(sc.arrays(), cam, 0.5, ost)
    n_gpu, n_rect, n_need = check_culled_binning(b, pre, ost, 256, 256, *tile)
    assert n_gpu <= 1.02 * n_need + 16, (n_gpu, n_need)
    assert n_gpu < 0.95 * n_rect, (n_gpu, n_rect)
    ctx.release(st)
    cfg0 = _lib.default_cfg(temporal_cull=cull, tile_w=tile[0], tile_h=tile[1], tile_cull=0)
    rgb0, _, _ = ctx.render(model, cam, 0.5, cfg0)
    assert torch.equal(rgb, rgb0)
    compare_image(rgb.cpu().numpy(), oc.composite(pre, cam, ost, mode="rect"))


def test_depth_ties_ordered_by_position(ctx):
    # several Gaussians share an exact depth (same mean); order must follow index
    sc = inputs.tiny_scene(300, seed=3)
    sc.log_scale[:3] += 1.2
    sc.mean[:, 100:140] = sc.mean[:, 100:101]
    sc.log_scale[:, 100:140] = sc.log_scale[:, 100:101]
    sc.q_left[:, 100:140] = sc.q_left[:, 100:101]
    sc.q_right[:, 100:140] = sc.q_right[:, 100:101]
    cam = inputs.look_at_camera(0.0, 3.0, 64, 64)
    rgb, _, st = ctx.render(to_dev(sc), cam, float(sc.mean[3, 100]), _lib.default_cfg(tile_cull=0),
                            keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    pre = oc.prepare(sc.arrays(), cam, float(sc.mean[3, 100]), oracle_settings())
    ids, _, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, 64, 64, 16, 16)
    assert np.array_equal(b["sorted_ids"].cpu().numpy().astype(np.uint32), ids)
    assert_same_ranges(b["tile_ranges"].cpu().numpy().astype(np.uint32), ranges)
    ref = oc.composite(pre, cam, oracle_settings(), mode="brute")
    compare_image(rgb.cpu().numpy(), ref)
    ctx.release(st)


def test_many_equal_depths_sorted_through_merges(ctx):
    """5000 of 6000 Gaussians share one exact depth: their depth bucket is
    larger than one LDS sort, so it is sorted in chunks and merged; the tile
    lists must still follow (depth, index) exactly."""
    sc = inputs.tiny_scene(6000, seed=5)
    sc.mean[:, 500:5500] = sc.mean[:, 500:501]
    sc.log_scale[:, 500:5500] = sc.log_scale[:, 500:501]
    sc.q_left[:, 500:5500] = sc.q_left[:, 500:501]
    sc.q_right[:, 500:5500] = sc.q_right[:, 500:501]
    sc.opacity_logit[500:5500] = -3.0
    cam = inputs.look_at_camera(10.0, 3.0, 48, 40)
    t = float(sc.mean[3, 500])
    _, _, st = ctx.render(to_dev(sc), cam, t, _lib.default_cfg(tile_cull=0), keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    pre = oc.prepare(sc.arrays(), cam, t, oracle_settings())
    assert pre.visible[500:5500].all()
    ids, _, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, 48, 40, 16, 16)
    assert np.array_equal(b["sorted_ids"].cpu().numpy().astype(np.uint32), ids)
    assert_same_ranges(b["tile_ranges"].cpu().numpy().astype(np.uint32), ranges)
    ctx.release(st)


def test_long_tile_lists_take_the_searched_ranges(ctx):
    """A 32x32 image (4 tiles) under 20000 enlarged Gaussians: thousands of
    instances per tile, so the ranges come from binary searches instead of key
    boundaries; lists and ranges must still match the oracle bit for bit."""
    sc = inputs.tiny_scene(20_000, seed=6)
    sc.log_scale[:3] += 1.5
    cam = inputs.look_at_camera(-5.0, 3.0, 32, 32)
    _, _, st = ctx.render(to_dev(sc), cam, 0.5, _lib.default_cfg(tile_cull=0), keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    pre = oc.prepare(sc.arrays(), cam, 0.5, oracle_settings())
    ids, _, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, 32, 32, 16, 16)
    assert ids.size > 2048 * 4
    assert np.array_equal(b["sorted_ids"].cpu().numpy().astype(np.uint32), ids)
    assert_same_ranges(b["tile_ranges"].cpu().numpy().astype(np.uint32), ranges)
    ctx.release(st)


@pytest.mark.parametrize("grow", [1.6, 2.3])
def test_many_instances_bin_exactly(ctx, grow):
    """8M and 19M instances (8x8 tiles, no tile culling): the tile sort takes
    4096 keys per block, two emission windows per block writing its first
    histogram, over thousands of histogram columns; lists and ranges must
    match the oracle bit for bit."""
    sc = inputs.tiny_scene(40_000, seed=8)
    sc.log_scale[:3] += grow
    sc.log_scale[3] += 3.0
    cam = inputs.look_at_camera(10.0, 3.0, 320, 240)
    cfg = _lib.default_cfg(tile_w=8, tile_h=8, tile_cull=0)
    _, _, st = ctx.render(to_dev(sc), cam, 0.5, cfg, keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    pre = oc.prepare(sc.arrays(), cam, 0.5, oracle_settings(cfg))
    ids, _, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, 320, 240, 8, 8)
    assert ids.size > (1 << 21) if grow < 2 else ids.size > 4096 * 4096
    assert b["n_inst"] == ids.size
    assert np.array_equal(b["sorted_ids"].cpu().numpy().astype(np.uint32), ids)
    assert_same_ranges(b["tile_ranges"].cpu().numpy().astype(np.uint32), ranges)
    ctx.release(st)


def assert_same_ranges(got, ref):
    """Non-empty tiles must match exactly; an empty tile may be any [s, s)."""
    nonempty = ref[:, 1] > ref[:, 0]
    bad = np.flatnonzero(nonempty & np.any(got != ref, axis=1))
    assert bad.size == 0, f"{bad.size} tiles differ, first {bad[:5]}"
    assert np.all(got[~nonempty, 0] == got[~nonempty, 1]), "an empty tile has a non-empty range"


# invariances -------------------------------------------------------------------------
def test_tile_and_batch_configs_give_identical_images(ctx):
    sc = inputs.tiny_scene(10_000, seed=0)
    cam = inputs.look_at_camera(0.0, 3.0, 200, 150)
    model = to_dev(sc)
    base = None
    for tile in ((16, 16), (8, 8), (32, 8), (32, 16), (32, 32)):
        for batch in ((64, 128, 256, 512, 1024) if tile == (32, 32) else (64, 128, 256)):
            for cull in (1, 0):
                for ppt, tcull, sched in ((1, 1, 1), (2, 1, 0), (4, 1, 1), (2, 0, 1), (1, 0, 0)):
                    cfg = _lib.default_cfg(tile_w=tile[0], tile_h=tile[1], batch=batch, temporal_cull=cull,
                                           pixels_per_thread=ppt, tile_cull=tcull, schedule=sched)
                    rgb, _, _ = ctx.render(model, cam, 0.5, cfg)
                    if base is None:
                        base = rgb.clone()
                    else:
                        diff = (rgb - base).abs()
                        assert torch.equal(rgb, base), (tile, batch, cull, ppt, tcull, sched, int((diff > 0).sum()),
                                                        float(diff.max()))


def test_forward_is_deterministic(ctx):
    sc = inputs.long_scene(20_000, seed=1)
    cam = inputs.arc_cameras(20, 4.0, 320, 240)[7]
    model = to_dev(sc)
    a, _, sa = ctx.render(model, cam, 0.3, keep_state=True)
    ba = ctx.binning(sa)
    b, _, sb = ctx.render(model, cam, 0.3, keep_state=True)
    bb = ctx.binning(sb)
    assert torch.equal(a, b)
    assert torch.equal(ba["sorted_ids"], bb["sorted_ids"]) and torch.equal(ba["tile_ranges"], bb["tile_ranges"])
    ctx.release(sa)
    ctx.release(sb)


def test_fixed_capacity_and_overflow(ctx):
    sc = inputs.tiny_scene(10_000, seed=0)
    cam = inputs.look_at_camera(0.0, 3.0, 256, 256)
    model = to_dev(sc)
    ref, _, st = ctx.render(model, cam, 0.5, keep_state=True)
    m = ctx.binning(st)["n_inst"]
    ctx.release(st)
    ctx.check_overflow()
    big, _, _ = ctx.render(model, cam, 0.5, _lib.default_cfg(instance_capacity=m + 1000))
    ctx.check_overflow()
    assert torch.equal(big, ref)
    ctx.render(model, cam, 0.5, _lib.default_cfg(instance_capacity=max(1, m // 2)))
    with pytest.raises(_lib.FdgsError) as e:
        ctx.check_overflow()
    assert e.value.code == _lib.FDGS_ERR_CAPACITY
    ctx.check_overflow()   # flag cleared


# a1 masks ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, 1])
def test_active_mask_bit_exact(ctx, mode):
    sc = inputs.long_scene(30_000, seed=2)
    views = inputs.arc_cameras(5, 4.0, 338, 254)
    frames = inputs.frame_times(300)[110:121]
    bits, idx, count = ctx.build_active_mask(to_dev(sc), frames, frames[0], frames[-1], mode, views)
    torch.cuda.synchronize()
    keep, rbits, ridx = omask.active_mask(sc.arrays(), frames, frames[0], frames[-1], mode, views,
                                          dilation=float(np.float32(0.3)), alpha_min=float(np.float32(1 / 255)))
    n = int(count.item())
    assert n == ridx.size
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), rbits)
    assert np.array_equal(idx[:n].cpu().numpy().view(np.uint32), ridx)


def test_temporal_mask_render_identical_to_dense(ctx):
    sc = inputs.long_scene(40_000, seed=5)
    cam = inputs.arc_cameras(20, 4.0, 338, 254)[3]
    model = to_dev(sc)
    frames = inputs.frame_times(300)[60:71]
    bits, idx, count = ctx.build_active_mask(model, frames, frames[0], frames[-1], 0)
    assert 0 < int(count.item()) < sc.n
    for f in (0, 4, 10):
        t = float(frames[f])
        dense, _, _ = ctx.render(model, cam, t)
        masked, _, _ = ctx.render(model, cam, t, idx=idx, n_idx=count)
        assert torch.equal(dense, masked)


# full-size parity ----------------------------------------------------------------------
# Launch configurations the benchmark's autotuner picks at 1352x1014 (tile,
# LDS batch, pixels per thread, schedule), besides the default one.
BENCH_CONFIGS = (((32, 32), 1024, 2, 1), ((32, 32), 512, 2, 1), ((32, 32), 256, 2, 1), ((32, 32), 128, 2, 1),
                 ((32, 16), 256, 2, 1), ((32, 16), 128, 2, 1), ((32, 32), 256, 2, 0), ((32, 16), 256, 2, 0),
                 ((16, 16), 256, 2, 0), ((32, 32), 1024, 2, 0))


@pytest.mark.parametrize("f,c", [(137, 11), (5, 0)])
def test_full_resolution_masked_frame_whole_image(ctx, f, c):
    """The headline workload (200k long-lived Gaussians, keyframe-window mask
    with the tile test, 1352x1014): every pixel against the oracle, in the
    default configuration; the benchmark's launch configurations give the same
    frame bit for bit."""
    sc = inputs.long_scene(200_000, seed=0)
    cams = inputs.arc_cameras(20, 4.0, 1352, 1014)
    model = to_dev(sc)
    frames = inputs.frame_times(300)
    keys, windows, fw = inputs.keyframe_windows(300, 10)
    lo, hi = windows[fw[f]]
    win = frames[lo:hi + 1]
    bits, idx, count = ctx.build_active_mask(model, win, frames[lo], frames[hi], 1, cams)
    cam = cams[c]
    t = float(frames[f])
    rgb, _, _ = ctx.render(model, cam, t, idx=idx, n_idx=count)
    torch.cuda.synchronize()
    n = int(count.item())
    sel = idx[:n].cpu().numpy().view(np.uint32).astype(np.int64)
    ref = oc.render(sc.arrays(), cam, t, oracle_settings(), idx=sel, mode="rect")
    worst, nflag = compare_image(rgb.cpu().numpy(), ref, label=f"masked 1352x1014 frame {f} camera {c}")
    print(f"1352x1014 masked frame {f}, camera {c}: {n}/{sc.n} kept, max err {worst:.2e}, flagged {nflag} "
          f"({nflag / ref.flags.size:.2e})")
    for tile, batch, ppt, sched in BENCH_CONFIGS:
        cfg = _lib.default_cfg(tile_w=tile[0], tile_h=tile[1], batch=batch, pixels_per_thread=ppt, schedule=sched,
                               instance_capacity=1 << 22)
        other, _, _ = ctx.render(model, cam, t, cfg, idx=idx, n_idx=count)
        assert torch.equal(other, rgb), (tile, batch, ppt, sched)
    ctx.check_overflow()


def test_single_view_above_bucket_limit_matches_oracle(ctx):
    """One view of more than 2^20 processed Gaussians takes the radix depth
    order instead of the depth buckets: lists and ranges bit for bit, and the
    whole image against the oracle (about 0.9M visible, 2M instances on 30
    tiles).  Some Gaussians sit 0.2 in front of the camera and cross the
    image as needles centred thousands of pixels away (the float32 exponent
    must not lose digits there).  A pixel here walks well over a thousand list
    entries before it saturates, so the allowed share of flagged pixels scales
    with its list entries per pixel as the default one does (225 per pixel)."""
    sc = inputs.tiny_scene(1_100_000, seed=9)
    sc.log_scale[3] += 3.0
    assert sc.n > (1 << 20)
    cam = inputs.look_at_camera(20.0, 3.0, 96, 72)
    cfg = _lib.default_cfg(tile_w=16, tile_h=16, tile_cull=0)
    rgb, _, st = ctx.render(to_dev(sc), cam, 0.5, cfg, keep_state=True)
    b = ctx.binning(st)
    torch.cuda.synchronize()
    ost = oracle_settings(cfg)
    pre = oc.prepare(sc.arrays(), cam, 0.5, ost)
    assert int(pre.visible.sum()) > 800_000
    ids, _, ranges = obin.bin_gaussians(pre.rect, pre.depth, pre.visible, 96, 72, 16, 16)
    assert b["n_inst"] == ids.size
    assert np.array_equal(b["sorted_ids"].cpu().numpy().astype(np.uint32), ids)
    assert_same_ranges(b["tile_ranges"].cpu().numpy().astype(np.uint32), ranges)
    ctx.release(st)
    ref = oc.composite(pre, cam, ost, mode="rect")
    # list entries per pixel (an upper bound on the entries a pixel evaluates)
    lens = np.diff(ranges.astype(np.int64), axis=1).reshape(-1)
    rows = np.minimum(16, 72 - 16 * (np.arange(lens.size) // 6))
    walked = float((lens * 16 * rows).sum()) / (96 * 72)
    worst, nflag = compare_image(rgb.cpu().numpy(), ref, max_flagged=MAX_FLAGGED_FRAC * max(1.0, walked / 225.0),
                                 label="1.1M needles 96x72")
    print(f"single view, {sc.n} Gaussians, {ids.size} instances: max err {worst:.2e}, flagged {nflag}")


def test_full_resolution_dense_frame_sampled(ctx):
    """The unfiltered 3M-Gaussian frame at 1352x1014 in the benchmark's
    configuration (no temporal or tile culling): 4096 seeded pixels plus every
    pixel of 8 seeded 16x16 tiles (one of them on the ragged bottom row)."""
    sc = inputs.dense_scene(3_000_000, seed=0)
    cams = inputs.arc_cameras(20, 4.0, 1352, 1014)
    t = float(inputs.frame_times(300)[123])
    cfg = _lib.default_cfg(temporal_cull=0, tile_cull=0)
    model = to_dev(sc)
    rgb, _, _ = ctx.render(model, cams[5], t, cfg)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    px = rng.integers(0, 1352, 4096)
    py = rng.integers(0, 1014, 4096)
    tiles_x, tiles_y = 1352 // 16 + 1, 1014 // 16 + 1          # 85 x 64, the last row 6 pixels high
    picks = list(rng.choice(tiles_x * (tiles_y - 1), 7, replace=False)) + [tiles_x * (tiles_y - 1) + 40]
    ty, tx = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    for tid in picks:
        gy, gx = divmod(int(tid), tiles_x)
        xs, ys = gx * 16 + tx.ravel(), gy * 16 + ty.ravel()
        keep = (xs < 1352) & (ys < 1014)
        px = np.concatenate([px, xs[keep]])
        py = np.concatenate([py, ys[keep]])
    ref = oc.render(sc.arrays(), cams[5], t, oracle_settings(cfg), mode="rect", pixels=(px, py))
    worst, nflag = compare_image(rgb.cpu().numpy(), ref, pixels=(px, py), label="dense 3M 1352x1014 sampled")
    print(f"1352x1014 dense frame: {px.size} pixels, max err {worst:.2e}, flagged {nflag}")


@pytest.mark.parametrize("dilation", [0.3, 0.0])
def test_tile_cull_keeps_images_on_anisotropic_scenes(ctx, dilation):
    """Elongated, rotated footprints up to and past the condition number at
    which culling falls back to the rectangle: the image with culling is the
    image without it, bit for bit."""
    cam = inputs.look_at_camera(10.0, 3.0, 300, 220)
    for k, stretch in enumerate((1.0, 3.0, 5.0, 7.0)):
        sc = inputs.tiny_scene(6000, seed=20 + k)
        sc.log_scale[k % 3] += stretch
        sc.log_scale[(k + 1) % 3] -= 1.0
        model = to_dev(sc)
        for cull in (1, 0):
            cfg1 = _lib.default_cfg(temporal_cull=cull, dilation=dilation)
            cfg0 = _lib.default_cfg(temporal_cull=cull, dilation=dilation, tile_cull=0)
            a, Ta, sa = ctx.render(model, cam, 0.5, cfg1, want_T=True, keep_state=True)
            b, Tb, _ = ctx.render(model, cam, 0.5, cfg0, want_T=True)
            n1 = ctx.binning(sa)["n_inst"]
            ctx.release(sa)
            assert torch.equal(a, b) and torch.equal(Ta, Tb), (stretch, cull)
            print(f"stretch {stretch} cull {cull}: {n1} instances with tile culling")


def test_tile_cull_keeps_full_resolution_frames(ctx):
    """The benchmark's scene and cameras at 1352x1014: identical frames with
    and without tile culling, and fewer instances."""
    sc = inputs.long_scene(200_000, seed=0)
    cams = inputs.arc_cameras(20, 4.0, 1352, 1014)
    model = to_dev(sc)
    for c, t in ((0, 0.1), (5, 0.5), (13, 0.77), (19, 0.95)):
        a, _, sa = ctx.render(model, cams[c], t, keep_state=True)
        b, _, sb = ctx.render(model, cams[c], t, _lib.default_cfg(tile_cull=0), keep_state=True)
        na, nb = ctx.binning(sa)["n_inst"], ctx.binning(sb)["n_inst"]
        ctx.release(sa)
        ctx.release(sb)
        assert torch.equal(a, b), (c, t)
        assert na < nb
        print(f"camera {c} t {t}: {na} instances with tile culling, {nb} without")


def test_contributed_mask_matches_oracle_and_keeps_keyframe_images(ctx):
    """Keyframe visibility (mode 2): the GPU set holds every Gaussian the
    FP64 oracle surely sees blended and only ones it may see blended, and a
    masked render of a mask view at a keyframe equals the dense render."""
    sc = inputs.long_scene(30_000, seed=3)
    views = inputs.arc_cameras(4, 4.0, 200, 150)
    model = to_dev(sc)
    t_lo, t_hi = 0.3, 0.333
    bits, idx, count = ctx.build_active_mask(model, [], t_lo, t_hi, _lib.MASK_CONTRIBUTED, views)
    torch.cuda.synchronize()
    n = int(count.item())
    got = np.zeros(sc.n, dtype=bool)
    got[idx[:n].cpu().numpy().view(np.uint32)] = True
    unpacked = ((bits.cpu().numpy().view(np.uint32)[:, None] >> np.arange(32, dtype=np.uint32)) & 1)
    assert np.array_equal(unpacked.astype(bool).ravel()[:sc.n], got)
    sure, maybe = omask.contributed_keep(sc.arrays(), views, (t_lo, t_hi), oracle_settings())
    assert np.all(got[sure]), int((sure & ~got).sum())
    assert np.all(maybe[got]), int((got & ~maybe).sum())
    assert 0 < n < sc.n
    for t in (t_lo, t_hi):
        for cam in views[::3]:
            dense, Td, _ = ctx.render(model, cam, t, want_T=True)
            masked, Tm, _ = ctx.render(model, cam, t, idx=idx, n_idx=count, want_T=True)
            assert torch.equal(dense, masked) and torch.equal(Td, Tm)
    print(f"contributed mask: {n} of {sc.n} kept; oracle sure {int(sure.sum())}, maybe {int(maybe.sum())}")


def test_frames_in_flight_on_four_streams_match_one(ctx):
    """Four contexts rendering consecutive frames round-robin on four streams
    at once (the benchmark's frame loop) give every frame bit for bit as one
    context does."""
    from paper_2503_16422_amd.render import Context
    sc = inputs.tiny_scene(20_000, seed=11)
    model = to_dev(sc)
    cams = [inputs.look_at_camera(10.0 * k, 3.0, 200, 150) for k in range(4)]
    times = [0.1, 0.35, 0.6, 0.85, 0.2, 0.7, 0.45, 0.95]
    cfg = _lib.default_cfg(tile_w=32, tile_h=32, batch=1024, schedule=1, instance_capacity=1 << 22)
    ref = [ctx.render(model, cams[k % 4], t, cfg)[0].clone() for k, t in enumerate(times)]
    others = [Context(0) for _ in range(3)]
    ctxs = [ctx] + others
    streams = [torch.cuda.Stream() for _ in ctxs]
    outs = torch.empty((len(times), 3, 150, 200), device="cuda")
    torch.cuda.synchronize()
    for k, t in enumerate(times):
        j = k % len(ctxs)
        with torch.cuda.stream(streams[j]):
            ctxs[j].render(model, cams[k % 4], t, cfg, out_rgb=outs[k])
    torch.cuda.synchronize()
    for c in others:
        c.check_overflow()
        c.close()
    for k in range(len(times)):
        assert torch.equal(outs[k], ref[k]), k


def test_headline_frames_in_flight_on_four_streams_match_one(ctx):
    """The benchmark's frame loop at full size: masked 1352x1014 frames of the
    200k-Gaussian scene dealt round-robin to four contexts on four streams,
    in a launch configuration the benchmark picks (32x32 tiles, LDS batch 512,
    longest list first), equal the one-context frames bit for bit."""
    from paper_2503_16422_amd.render import Context
    sc = inputs.long_scene(200_000, seed=0)
    cams = inputs.arc_cameras(20, 4.0, 1352, 1014)
    model = to_dev(sc)
    frames = inputs.frame_times(300)
    keys, windows, fw = inputs.keyframe_windows(300, 10)
    picks = [(40, 2), (41, 9), (42, 17), (43, 3), (44, 12), (45, 19), (46, 6), (47, 14)]
    masks = {}
    for f, _ in picks:
        w = fw[f]
        if w not in masks:
            lo, hi = windows[w]
            _, idx, count = ctx.build_active_mask(model, frames[lo:hi + 1], frames[lo], frames[hi], 1, cams)
            masks[w] = (idx, count)
    cfg = _lib.default_cfg(tile_w=32, tile_h=32, batch=512, pixels_per_thread=2, schedule=1,
                           instance_capacity=1 << 22)
    ref = []
    for f, c in picks:
        idx, count = masks[fw[f]]
        ref.append(ctx.render(model, cams[c], float(frames[f]), cfg, idx=idx, n_idx=count)[0].clone())
    others = [Context(0) for _ in range(3)]
    ctxs = [ctx] + others
    streams = [torch.cuda.Stream() for _ in ctxs]
    outs = torch.empty((len(picks), 3, 1014, 1352), device="cuda")
    torch.cuda.synchronize()
    for k, (f, c) in enumerate(picks):
        j = k % len(ctxs)
        idx, count = masks[fw[f]]
        with torch.cuda.stream(streams[j]):
            ctxs[j].render(model, cams[c], float(frames[f]), cfg, idx=idx, n_idx=count, out_rgb=outs[k])
    torch.cuda.synchronize()
    for c in ctxs:
        c.check_overflow()
    for c in others:
        c.close()
    for k in range(len(picks)):
        assert torch.equal(outs[k], ref[k]), picks[k]


def test_active_ratio_and_activation_iou(ctx):
    """The redundancy measures of Sec. 4.1 from contributed masks at single
    timestamps: fdgs_mask_overlap counts bit-exactly (on the oracle's own sets,
    uploaded, and on the GPU's), and the GPU's active sets lie between the
    oracle's sure and possible sets (a ragged n exercises the last word)."""
    sc = inputs.long_scene(29_999, seed=3)
    views = inputs.arc_cameras(4, 4.0, 200, 150)
    model = to_dev(sc)
    st = oracle_settings()
    n = sc.n
    sets = {}
    for t in (0.3, 0.5):
        bits, idx, count = ctx.build_active_mask(model, [], t, t, _lib.MASK_CONTRIBUTED, views)
        sure, maybe = omask.contributed_keep(sc.arrays(), views, (t,), st)
        got = np.zeros(n, dtype=bool)
        got[idx[:int(count.item())].cpu().numpy().view(np.uint32)] = True
        assert np.all(got[sure]) and np.all(maybe[got])
        sets[t] = (bits, got, sure, maybe)
    (b0, g0, s0, m0), (b1, g1, s1, m1) = sets[0.3], sets[0.5]
    out = ctx.mask_overlap(b0, b1, n).cpu().numpy()
    assert list(out) == [int(g0.sum()), int(g1.sum()), int((g0 & g1).sum())]
    # the counting kernel on the oracle's sets, uploaded
    dev = lambda keep: torch.from_numpy(omask.pack_bits(keep).view(np.int32)).cuda()
    for a, b in ((s0, s1), (m0, m1), (s0, m1)):
        out = ctx.mask_overlap(dev(a), dev(b), n).cpu().numpy()
        assert list(out) == [int(a.sum()), int(b.sum()), int((a & b).sum())]
    ratio = g1.sum() / n
    iou = (g0 & g1).sum() / (g0 | g1).sum()
    assert s1.sum() / n <= ratio <= m1.sum() / n
    assert 0.0 < iou < 1.0
    print(f"active ratio at t=0.5: {ratio:.4f} (oracle {s1.sum() / n:.4f}..{m1.sum() / n:.4f}); "
          f"IoU(0.3, 0.5) {iou:.4f}")
