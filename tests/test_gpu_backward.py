"""GPU adjoint (render_backward) against the FP64 torch-autograd oracle."""
import numpy as np
import pytest
import torch

from oracle import grad as og
from paper_2503_16422_amd import _lib, inputs
from tests.gpu_helpers import oracle_settings

pytestmark = pytest.mark.gpu

NAMES = ["mean", "log_scale", "q_left", "q_right", "opacity_logit", "sh"]


@pytest.fixture(scope="module")
def ctx():
    from paper_2503_16422_amd.render import Context
    c = Context(0)
    yield c
    c.close()


def rel_err(g, r):
    return float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30))


def check_grads(gpu, ref, tol=1e-3):
    errs = {}
    for k in NAMES:
        g = gpu[k].detach().cpu().numpy().astype(np.float64)
        r = ref[k]
        errs[k] = rel_err(g, r)
        assert errs[k] <= tol, (k, errs[k])
        # elementwise, relative to the tensor's scale
        assert np.all(np.abs(g - r) <= tol * (np.abs(r) + 1e-3 * np.abs(r).max()) + 1e-12), k
    return errs


def same_up_to_atomic_order(a, b):
    """Two runs of the same adjoint differ only in the order of the float
    atomics that add pixel contributions into the 2D gradients.  A repeated
    run on one stream already moves single elements by up to 1e-4 of their
    own size, or 6e-7 of the tensor's largest element, so the bound is ten
    times that; a view dropped or added twice moves whole gradients."""
    return torch.allclose(a, b, rtol=1e-4, atol=1e-5 * float(b.abs().max()) + 1e-12)


def scene_small(n, seed, grow=1.0):
    sc = inputs.dense_scene(n, seed=seed)
    sc.log_scale[:3] += grow
    sc.log_scale[3] = np.float32(-1.0)
    return sc


@pytest.mark.parametrize("n,size,grow,tile,batch,ppt", [(64, 32, 1.0, (16, 16), 128, 2),
                                                        (2000, 128, 0.5, (16, 16), 128, 2),
                                                        (2000, 128, 0.5, (32, 16), 128, 2),
                                                        (2000, 128, 0.5, (32, 32), 128, 2),
                                                        (2000, 128, 0.5, (32, 32), 1024, 2),
                                                        (2000, 128, 0.5, (8, 8), 128, 1),
                                                        (2000, 128, 0.5, (16, 16), 256, 4),
                                                        (2000, 128, 0.5, (32, 16), 256, 4),
                                                        (2000, 128, 0.5, (32, 8), 128, 4),
                                                        (2000, 100, 0.5, (32, 32), 256, 4)])
def test_backward_matches_oracle_gradient(ctx, n, size, grow, tile, batch, ppt):
    """The adjoint takes 2 or 4 pixels per thread after the forward's (1 for
    8x8 tiles); the 100x100 image leaves ragged tiles."""
    from paper_2503_16422_amd.render import GaussianModel
    sc = scene_small(n, seed=3, grow=grow)
    cam = inputs.look_at_camera(0.0, 3.0, size, size)
    cfg = _lib.default_cfg(bg=(0.1, 0.2, 0.3), tile_w=tile[0], tile_h=tile[1], batch=batch, pixels_per_thread=ppt)
    model = GaussianModel.from_scene(sc, "cuda:0")
    rgb, _, state = ctx.render(model, cam, 0.5, cfg, keep_state=True)
    G = np.random.default_rng(0).standard_normal((3, size, size))
    grads = ctx.backward(state, torch.from_numpy(G.astype(np.float32)).cuda(), model)
    torch.cuda.synchronize()
    ctx.release(state)
    ref = og.render_vjp(sc.arrays(), cam, 0.5, oracle_settings(cfg), G)
    errs = check_grads(grads, ref)
    print(f"n={n}: relative errors " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))


def test_masked_backward_scatters_to_model_layout(ctx):
    from paper_2503_16422_amd.render import GaussianModel
    sc = scene_small(600, seed=5, grow=0.7)
    cam = inputs.look_at_camera(15.0, 3.0, 64, 48)
    model = GaussianModel.from_scene(sc, "cuda:0")
    keep = np.sort(np.random.default_rng(2).choice(sc.n, 350, replace=False))
    idx = torch.from_numpy(keep.astype(np.int32)).cuda()
    n_idx = torch.tensor([keep.size], dtype=torch.int64, device="cuda")
    rgb, _, state = ctx.render(model, cam, 0.5, idx=idx, n_idx=n_idx, keep_state=True)
    G = np.random.default_rng(1).standard_normal((3, 48, 64))
    grads = ctx.backward(state, torch.from_numpy(G.astype(np.float32)).cuda(), model)
    torch.cuda.synchronize()
    ctx.release(state)
    ref_sub = og.render_vjp(sc.subset(keep).arrays(), cam, 0.5, oracle_settings(), G)
    dropped = np.setdiff1d(np.arange(sc.n), keep)
    for k in NAMES:
        g = grads[k].detach().cpu().numpy()
        assert np.all(g[..., dropped] == 0), k
    sub = {k: grads[k][..., torch.from_numpy(keep).cuda()] for k in NAMES}
    check_grads(sub, ref_sub)


def test_autograd_function_matches_direct_call(ctx):
    from paper_2503_16422_amd.render import GaussianModel, Render4DGS
    sc = scene_small(300, seed=7, grow=0.8)
    cam = inputs.look_at_camera(-20.0, 3.0, 48, 48)
    model = GaussianModel.from_scene(sc, "cuda:0")
    params = [t.clone().requires_grad_(True) for t in model.tensors()]
    cfg = _lib.default_cfg()
    target = torch.rand(3, 48, 48, device="cuda")
    rgb = Render4DGS.apply(ctx, cam, 0.45, cfg, None, None, *params)
    loss = 0.5 * ((rgb - target) ** 2).sum()
    loss.backward()
    rgb2, _, state = ctx.render(model, cam, 0.45, cfg, keep_state=True)
    assert torch.equal(rgb.detach(), rgb2)
    direct = ctx.backward(state, (rgb2 - target).contiguous(), model)
    ctx.release(state)
    for p, k in zip(params, NAMES):
        assert same_up_to_atomic_order(p.grad, direct[k]), k


def crop_camera(cam, x0, y0, w, h):
    """The same pinhole restricted to pixels [x0, x0 + w) x [y0, y0 + h)."""
    c = inputs.Camera(cam.R, cam.tvec, cam.fx, cam.fy, cam.cx - x0, cam.cy - y0, w, h, cam.znear)
    return c


@pytest.mark.parametrize("crop", [(600, 480), (1320, 990)])
def test_backward_full_scene_on_crops(ctx, crop):
    """500k-Gaussian scene, 1352x1014 camera: the gradient of a 32x32 crop.
    Gaussians whose footprint misses the crop contribute nothing, so the
    oracle differentiates only the ones that reach it."""
    from oracle import composite as oc
    from paper_2503_16422_amd.render import GaussianModel
    sc = inputs.dense_scene(500_000, seed=0)
    cam = crop_camera(inputs.arc_cameras(20, 4.0, 1352, 1014)[5], crop[0], crop[1], 32, 32)
    t = 0.6001
    model = GaussianModel.from_scene(sc, "cuda:0")
    rgb, _, state = ctx.render(model, cam, t, keep_state=True)
    G = np.random.default_rng(3).standard_normal((3, 32, 32))
    grads = ctx.backward(state, torch.from_numpy(G.astype(np.float32)).cuda(), model)
    torch.cuda.synchronize()
    ctx.release(state)
    st = oracle_settings()
    pre = oc.prepare(sc.arrays(), cam, t, st)
    keep = np.flatnonzero(pre.visible)
    assert 0 < keep.size < 20_000
    ref = og.render_vjp(sc.subset(keep).arrays(), cam, t, st, G)
    sub = {k: grads[k][..., torch.from_numpy(keep).cuda()] for k in NAMES}
    errs = check_grads(sub, ref)
    drop = np.ones(sc.n, dtype=bool)
    drop[keep] = False
    dropped = torch.from_numpy(drop).cuda()
    for k in NAMES:
        assert torch.all(grads[k][..., dropped] == 0), k
    print(f"crop {crop}: {keep.size} Gaussians reach it; errors " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))


def test_views_pipelined_over_contexts_match_one_stream(ctx):
    """forward_backward_views over 1, 2 and 3 contexts (one stream each) adds
    the same gradients as the views rendered and differentiated one after
    another on one stream (up to the order of the adjoint's float atomics)."""
    from paper_2503_16422_amd.render import Context, GaussianModel, forward_backward_views
    sc = scene_small(3000, seed=11, grow=0.3)
    model = GaussianModel.from_scene(sc, "cuda:0")
    cams = inputs.arc_cameras(20, 4.0, 200, 150)
    keep = np.sort(np.random.default_rng(4).choice(sc.n, 2100, replace=False))
    idx = torch.from_numpy(keep.astype(np.int32)).cuda()
    n_idx = torch.tensor([keep.size], dtype=torch.int64, device="cuda")
    views = [(cams[c], t, i, n) for c, t, i, n in [(3, 0.2, None, None), (9, 0.5, idx, n_idx), (14, 0.71, None, None),
                                                    (1, 0.9, idx, n_idx), (17, 0.33, None, None)]]
    tgt = [torch.rand(3, 150, 200, device="cuda") for _ in views]
    cfg = _lib.default_cfg()
    ref = {k: torch.zeros_like(getattr(model, k)) for k in NAMES}
    for v, (cam, t, i, n) in enumerate(views):
        rgb, _, st = ctx.render(model, cam, t, cfg, idx=i, n_idx=n, keep_state=True)
        ctx.backward(st, rgb - tgt[v], model, ref)
        ctx.release(st)
    torch.cuda.synchronize()
    for n_ctx in (1, 2, 3):
        ctxs = [ctx] + [Context(0) for _ in range(n_ctx - 1)]
        got = {k: torch.zeros_like(getattr(model, k)) for k in NAMES}
        states = None
        for _ in range(2):   # the second pass reuses the states
            for g in got.values():
                g.zero_()
            states = forward_backward_views(ctxs, model, views, cfg, lambda v, rgb: rgb - tgt[v], got, states)
        torch.cuda.synchronize()
        for st in states:
            st.release()
        for c in ctxs[1:]:
            c.close()
        for k in NAMES:
            assert same_up_to_atomic_order(got[k], ref[k]), (n_ctx, k)


def test_backward_in_two_phases(ctx):
    """fdgs_render_backward_2d then fdgs_render_backward_params adds the same
    gradients as fdgs_render_backward (up to the order of float atomics); the
    second phase is refused on a state whose first phase has not run since its
    forward."""
    from paper_2503_16422_amd.render import GaussianModel
    sc = scene_small(1500, seed=13, grow=0.5)
    cam = inputs.look_at_camera(25.0, 3.0, 96, 80)
    model = GaussianModel.from_scene(sc, "cuda:0")
    rgb, _, state = ctx.render(model, cam, 0.55, keep_state=True)
    G = torch.from_numpy(np.random.default_rng(5).standard_normal((3, 80, 96)).astype(np.float32)).cuda()
    ref = ctx.backward(state, G, model)
    rgb, _, state = ctx.render(model, cam, 0.55, keep_state=state)
    with pytest.raises(_lib.FdgsError) as e:
        ctx.backward_params(state, model)
    assert e.value.code == _lib.FDGS_ERR_STATE
    ctx.backward_2d(state, G)
    got = ctx.backward_params(state, model)
    torch.cuda.synchronize()
    ctx.release(state)
    for k in NAMES:
        assert same_up_to_atomic_order(got[k], ref[k]), k
