"""Pins for the FP64 oracle: closed forms, textbook identities, invariants and
brute force, each chosen so that a plausible slip in the oracle (a dropped
term, a sign, a transposed operand, a wrong variance convention) fails one."""
import math

import numpy as np
import pytest
import torch

from oracle import binning, mask, optim, prune, sh as osh
from oracle import composite as oc
from oracle import grad as og
from oracle import slicing
from oracle.projection import project
from paper_2503_16422_amd import inputs

RNG = np.random.default_rng(1234)


def rand_quats(n, rng=RNG):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def left_matrix(q):
    a, b, c, d = q
    return np.array([[a, -b, -c, -d], [b, a, -d, c], [c, d, a, -b], [d, -c, b, a]])


def right_matrix(q):
    p, q_, r, s = q
    return np.array([[p, -q_, -r, -s], [q_, p, s, -r], [r, -s, p, q_], [s, r, -q_, p]])


def conj(q):
    return q * np.array([1.0, -1.0, -1.0, -1.0])


# P-1 quaternion algebra -----------------------------------------------------
def test_rotation_is_special_orthogonal_and_matches_products():
    ql, qr = rand_quats(64), rand_quats(64)
    R = slicing.rotation_4d(ql, qr)
    eye = np.eye(4)
    for k in range(64):
        assert np.allclose(R[k] @ R[k].T, eye, atol=1e-13)
        assert math.isclose(np.linalg.det(R[k]), 1.0, abs_tol=1e-12)
        # left/right multiplication matrices commute and compose to R
        L, Rm = left_matrix(ql[k]), right_matrix(qr[k])
        assert np.allclose(L @ Rm, Rm @ L, atol=1e-14)
        assert np.allclose(R[k], L @ Rm, atol=1e-14)
    # sign symmetry and identity
    assert np.allclose(slicing.rotation_4d(-ql, -qr), R, atol=1e-14)
    ident = np.tile([1.0, 0, 0, 0], (3, 1))
    assert np.allclose(slicing.rotation_4d(ident, ident), np.tile(eye, (3, 1, 1)))
    # unnormalised input is normalised first
    assert np.allclose(slicing.rotation_4d(3.0 * ql, 0.5 * qr), R, atol=1e-13)


def test_quaternion_product_is_hamilton():
    i = np.array([0.0, 1, 0, 0]); j = np.array([0.0, 0, 1, 0]); k = np.array([0.0, 0, 0, 1])
    assert np.allclose(slicing.quat_mul(i, j), k)
    assert np.allclose(slicing.quat_mul(j, k), i)
    assert np.allclose(slicing.quat_mul(k, i), j)
    assert np.allclose(slicing.quat_mul(i, i), [-1.0, 0, 0, 0])


# P-2 block-diagonal covariance reduces to a static 3D Gaussian ---------------
def block_diag_quats(n, rng=RNG):
    ql = rand_quats(n, rng)
    k = np.array([0.0, 0, 0, 1])
    qr = np.stack([slicing.quat_mul(slicing.quat_mul(conj(k), conj(q)), k) for q in ql])
    return ql, qr


def test_block_diagonal_reduces_to_3dgs():
    n = 32
    ql, qr = block_diag_quats(n)
    R = slicing.rotation_4d(ql, qr)
    assert np.allclose(R[:, :3, 3], 0, atol=1e-14) and np.allclose(R[:, 3, :3], 0, atol=1e-14)
    assert np.allclose(R[:, 3, 3], 1, atol=1e-14)
    log_s = RNG.normal(-3, 0.5, (n, 4))
    mean = RNG.uniform(-1, 1, (n, 4))
    s = np.exp(log_s)
    for t in (0.0, 0.3, 0.9):
        mean3, cov3, p = slicing.slice_at(mean, log_s, ql, qr, t)
        assert np.allclose(mean3, mean[:, :3], atol=1e-14)
        R3 = R[:, :3, :3]
        ref = np.einsum('nij,nj,nkj->nik', R3, s[:, :3] ** 2, R3)
        assert np.allclose(cov3, ref, rtol=1e-12, atol=1e-18)
        assert np.allclose(p, np.exp(-(t - mean[:, 3]) ** 2 / (2 * s[:, 3] ** 2)), rtol=1e-12)


# P-3 conditional formulas against independent identities --------------------
def test_conditional_matches_schur_and_density_ratio():
    n = 48
    ql, qr = rand_quats(n), rand_quats(n)
    log_s = RNG.normal(-2, 0.7, (n, 4))
    mean = RNG.uniform(-1, 1, (n, 4))
    t = 0.37
    mean3, cov3, p = slicing.slice_at(mean, log_s, ql, qr, t)
    Sigma = slicing.covariance_4d(log_s, ql, qr)
    P = np.linalg.inv(Sigma)
    for k in range(n):
        # precision-matrix form of the conditional
        c_ref = np.linalg.inv(P[k, :3, :3])
        assert np.allclose(cov3[k], c_ref, rtol=1e-7, atol=1e-14 * np.abs(c_ref).max())
        m_ref = mean[k, :3] - c_ref @ P[k, :3, 3] * (t - mean[k, 3])
        assert np.allclose(mean3[k], m_ref, rtol=1e-8, atol=1e-10)
        w = np.linalg.eigvalsh(cov3[k])
        assert w.min() >= -1e-12 * w.max()
        # the joint density at (x, t) divided by the conditional density at x is
        # the same for every x (it is the marginal density of t)
        xs = mean3[k] + RNG.standard_normal((5, 3)) * np.sqrt(np.diag(cov3[k]))
        ratio = []
        for x in xs:
            z4 = np.concatenate([x, [t]]) - mean[k]
            lj = -0.5 * z4 @ P[k] @ z4
            z3 = x - mean3[k]
            lc = -0.5 * z3 @ np.linalg.solve(cov3[k], z3)
            ratio.append(lj - lc)
        assert np.ptp(ratio) < 1e-6 * (1 + np.abs(ratio).max())
        # and that marginal is log p up to the normalising constants
        assert math.isclose(ratio[0] - 0.5 * math.log(np.linalg.det(Sigma[k]) / np.linalg.det(cov3[k]) / Sigma[k, 3, 3]),
                            math.log(p[k]), rel_tol=1e-6, abs_tol=1e-7)


def test_projector_form_and_minor_singular_values():
    n = 32
    ql, qr = rand_quats(n), rand_quats(n)
    log_s = RNG.normal(-2, 0.7, (n, 4))
    _, cov3, _ = slicing.slice_at(np.zeros((n, 4)), log_s, ql, qr, 0.0)
    R = slicing.rotation_4d(ql, qr)
    s = np.exp(log_s)
    for k in range(n):
        A = R[k, :3, :] * s[k]
        u = R[k, 3, :] * s[k]
        uh = u / np.linalg.norm(u)
        B = A @ (np.eye(4) - np.outer(uh, uh))
        assert np.allclose(B @ B.T, cov3[k], rtol=1e-9, atol=1e-15)
        sv = np.linalg.svd(R[k, :3, :3], compute_uv=False)
        assert np.allclose(sorted(sv), sorted([1.0, 1.0, abs(R[k, 3, 3])]), atol=1e-12)


# P-4 temporal marginal --------------------------------------------------------
def test_temporal_marginal_peak_and_second_derivative():
    n = 16
    ql, qr = rand_quats(n), rand_quats(n)
    log_s = RNG.normal(-2, 0.4, (n, 4))
    mean = RNG.uniform(0.2, 0.8, (n, 4))
    Sigma_t = slicing.covariance_4d(log_s, ql, qr)[:, 3, 3]
    for k in range(n):
        one = lambda tt: slicing.slice_at(mean[k:k + 1], log_s[k:k + 1], ql[k:k + 1], qr[k:k + 1], tt)[2][0]
        assert math.isclose(one(mean[k, 3]), 1.0, rel_tol=0, abs_tol=1e-15)
        t = mean[k, 3] + 0.7 * math.sqrt(Sigma_t[k])
        h = 1e-4 * math.sqrt(Sigma_t[k])
        d2 = (one(t + h) - 2 * one(t) + one(t - h)) / h ** 2
        eq5 = ((t - mean[k, 3]) ** 2 / Sigma_t[k] ** 2 - 1.0 / Sigma_t[k]) * one(t)
        assert math.isclose(d2, eq5, rel_tol=1e-5, abs_tol=1e-6 / Sigma_t[k])


# Small scenes used by the image pins -----------------------------------------
def scene_from_rows(mean, log_s, ql, qr, logit, sh):
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)
    return (f(mean), f(log_s), f(ql), f(qr), np.asarray(logit, dtype=np.float64),
            np.ascontiguousarray(np.transpose(np.asarray(sh, dtype=np.float64), (1, 2, 0))), 3)


def iso_gaussian(center, s, dc, logit, t_mean=0.5, log_st=-1.0):
    ql, qr = block_diag_quats(1)
    sh = np.zeros((1, 16, 3))
    sh[0, 0] = dc
    return ([list(center) + [t_mean]], [[math.log(s)] * 3 + [log_st]], ql, qr, [logit], sh)


def stack_scenes(*gs):
    parts = list(zip(*gs))
    return scene_from_rows(*(np.concatenate([np.asarray(p) for p in part]) for part in parts))


CAM = inputs.look_at_camera(0.0, 3.0, 64, 64)


# P-5 single isotropic Gaussian ------------------------------------------------
def test_single_isotropic_gaussian_analytic_image():
    s, D = 0.05, 3.0
    dc = np.array([0.6, -0.2, 1.5])
    g = iso_gaussian((0.0, 0.0, 0.0), s, dc, logit=0.8, t_mean=0.45, log_st=-1.5)
    scene = stack_scenes(g)
    st = oc.Settings(bg=(0.1, 0.2, 0.3))
    t = 0.5
    img = oc.render(scene, CAM, t, st, mode="brute")
    f = CAM.fx
    var = (f * s / D) ** 2 + st.dilation
    sigma = 1 / (1 + math.exp(-0.8))
    p = math.exp(-(t - 0.45) ** 2 / (2 * math.exp(-3.0)))
    c = np.maximum(0.0, dc / (2 * math.sqrt(math.pi)) + 0.5)
    py, px = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    r2 = (px + 0.5 - 32) ** 2 + (py + 0.5 - 32) ** 2
    alpha = np.minimum(0.99, sigma * p * np.exp(-r2 / (2 * var)))
    alpha = np.where(alpha < 1 / 255, 0.0, alpha)
    bg = np.array(st.bg)[:, None, None]
    expect = bg + alpha[None] * (c[:, None, None] - bg)
    assert np.abs(img.rgb - expect).max() < 1e-12
    assert np.abs(img.T - (1 - alpha)).max() < 1e-12


# P-6 two layers ----------------------------------------------------------------
def test_two_layer_closed_form_and_order():
    gA = iso_gaussian((0.0, 0.0, 0.3), 0.08, np.array([1.0, 0.0, 0.0]), 1.0)   # nearer (camera at z=3)
    gB = iso_gaussian((0.0, 0.0, -0.3), 0.08, np.array([0.0, 1.0, 0.0]), 0.5)
    st = oc.Settings(bg=(0.05, 0.05, 0.05))
    pix = (np.array([32, 30, 35]), np.array([32, 33, 29]))
    for scene in (stack_scenes(gA, gB), stack_scenes(gB, gA)):
        pre = oc.prepare(scene, CAM, 0.5, st)
        near = int(np.argmin(pre.depth))
        far = 1 - near
        img = oc.composite(pre, CAM, st, mode="brute", pixels=pix)
        for k in range(3):
            a = []
            for i in (near, far):
                dx = pix[0][k] + 0.5 - pre.uv[i, 0]
                dy = pix[1][k] + 0.5 - pre.uv[i, 1]
                ca, cb, cc = pre.conic[i]
                al = min(0.99, pre.opac[i] * math.exp(-0.5 * (ca * dx * dx + 2 * cb * dx * dy + cc * dy * dy)))
                a.append(al if al >= 1 / 255 else 0.0)
            expect = (pre.rgb[near] * a[0] + pre.rgb[far] * a[1] * (1 - a[0])
                      + np.array(st.bg) * (1 - a[0]) * (1 - a[1]))
            assert np.allclose(img.rgb[:, k], expect, atol=1e-14)
    # moving the far one in front changes the result
    gB2 = iso_gaussian((0.0, 0.0, 0.6), 0.08, np.array([0.0, 1.0, 0.0]), 0.5)
    a = oc.render(stack_scenes(gA, gB), CAM, 0.5, st, mode="brute", pixels=pix).rgb
    b = oc.render(stack_scenes(gA, gB2), CAM, 0.5, st, mode="brute", pixels=pix).rgb
    assert np.abs(a - b).max() > 1e-2


# P-7 transmittance --------------------------------------------------------------
def test_transmittance_bounds_and_monotone():
    sc = inputs.tiny_scene(3000, seed=5)
    cam = inputs.look_at_camera(0.0, 3.0, 48, 48)
    st = oc.Settings()
    pre = oc.prepare(sc.arrays(), cam, 0.5, st)
    img = oc.composite(pre, cam, st, mode="brute")
    assert img.T.min() >= st.t_min * (1 - st.alpha_max) - 1e-15
    assert img.T.max() <= 1.0
    assert img.rgb.min() >= 0.0
    # T along one pixel's walk never increases
    order = oc.depth_order(pre)
    px, py = 24, 24
    T = 1.0
    for i in order:
        dx, dy = px + 0.5 - pre.uv[i, 0], py + 0.5 - pre.uv[i, 1]
        a, b, c = pre.conic[i]
        al = min(st.alpha_max, pre.opac[i] * math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)))
        if al < st.alpha_min:
            continue
        if T * (1 - al) < st.t_min:
            break
        assert T * (1 - al) <= T
        T *= 1 - al
    assert math.isclose(T, img.T[py, px], rel_tol=1e-12)


# P-8 scale invariance -----------------------------------------------------------
def test_spatial_scale_invariance():
    rng = np.random.default_rng(7)
    n = 40
    ql, qr = block_diag_quats(n, rng)
    mean = np.concatenate([rng.uniform(-0.5, 0.5, (n, 3)), rng.uniform(0.3, 0.7, (n, 1))], 1)
    log_s = np.concatenate([rng.normal(-3, 0.3, (n, 3)), np.full((n, 1), -1.0)], 1)
    logit = rng.standard_normal(n)
    sh = rng.normal(0, 0.2, (n, 16, 3))
    st = oc.Settings()
    base = oc.render(scene_from_rows(mean, log_s, ql, qr, logit, sh), CAM, 0.5, st, mode="brute")
    kappa = 2.5
    m2 = mean.copy(); m2[:, :3] *= kappa
    ls2 = log_s.copy(); ls2[:, :3] += math.log(kappa)
    cam2 = inputs.look_at_camera(0.0, 3.0 * kappa, 64, 64)
    scaled = oc.render(scene_from_rows(m2, ls2, ql, qr, logit, sh), cam2, 0.5, st, mode="brute")
    assert np.abs(base.rgb - scaled.rgb).max() < 1e-9
    # shifting time and every mu_t together changes nothing either
    m3 = mean.copy(); m3[:, 3] += 0.25
    shifted = oc.render(scene_from_rows(m3, log_s, ql, qr, logit, sh), CAM, 0.75, st, mode="brute")
    assert np.abs(base.rgb - shifted.rgb).max() < 1e-9


# P-9 SH basis -------------------------------------------------------------------
def test_sh_basis_orthonormal_and_matches_formula():
    xg, wg = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = np.arange(nphi) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st_ = np.sqrt(1 - ct ** 2)
    d = np.stack([st_ * np.cos(ph), st_ * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).ravel()
    Y = osh.real_sh_basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)
    Yt = og.real_sh_basis(torch.as_tensor(d), 3).numpy()
    assert np.allclose(Yt, Y, atol=1e-12)
    # a couple of closed forms: Y_00 and Y_10 = sqrt(3/4pi) z
    assert np.allclose(Y[:, 0], 0.5 / math.sqrt(math.pi))
    assert np.allclose(Y[:, 2], math.sqrt(3 / (4 * math.pi)) * d[:, 2])


def test_sh_degree0_view_independent():
    rng = np.random.default_rng(3)
    sh = rng.normal(0, 0.3, (5, 16, 3))
    d = rng.standard_normal((5, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    d2 = rng.standard_normal((5, 3)); d2 /= np.linalg.norm(d2, axis=1, keepdims=True)
    assert np.allclose(osh.sh_color(sh, d, 0), osh.sh_color(sh, d2, 0))


# P-10 tiny brute force ------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5])
def test_tiny_scene_python_c_brute_rect_identical(n):
    sc = inputs.tiny_scene(n, seed=10 + n)
    sc.log_scale[:3] += 1.5          # make them cover some pixels of a 16x16 image
    sc.mean[3] = 0.5
    cam = inputs.look_at_camera(0.0, 3.0, 16, 16)
    st = oc.Settings(bg=(0.2, 0.1, 0.0))
    pre = oc.prepare(sc.arrays(), cam, 0.5, st)
    brute = oc.composite(pre, cam, st, mode="brute")
    rect = oc.composite(pre, cam, st, mode="rect")
    assert np.array_equal(brute.rgb, rect.rgb) and np.array_equal(brute.T, rect.T)
    order = oc.depth_order(pre)
    for py in range(16):
        for px in range(16):
            c, T = oc.composite_py(pre, order, px, py, st)
            assert np.array_equal(c, brute.rgb[:, py, px]) and T == brute.T[py, px]


def test_rect_mode_identical_to_brute_on_tiny_config():
    sc = inputs.tiny_scene(4000, seed=0)
    cam = inputs.look_at_camera(0.0, 3.0, 96, 96)
    for cull in (True, False):
        st = oc.Settings(temporal_cull=cull)
        pre = oc.prepare(sc.arrays(), cam, 0.5, st)
        a = oc.composite(pre, cam, st, mode="brute")
        b = oc.composite(pre, cam, st, mode="rect")
        assert np.array_equal(a.rgb, b.rgb) and np.array_equal(a.T, b.T)


# P-11 mask invariants ----------------------------------------------------------------
def test_temporal_mask_render_equals_dense_and_bits():
    sc = inputs.tiny_scene(6000, seed=2)
    cam = inputs.look_at_camera(20.0, 3.0, 64, 64)
    frames = inputs.frame_times(300)[40:51]
    keep, bits, idx = mask.active_mask(sc.arrays(), frames, frames[0], frames[-1], mask.TEMPORAL)
    assert 0 < keep.sum() < keep.size
    unpacked = ((bits[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(bool).ravel()[:keep.size]
    assert np.array_equal(unpacked, keep)
    assert np.array_equal(idx, np.flatnonzero(unpacked))
    st = oc.Settings()
    for t in (frames[0], frames[4], frames[-1]):
        dense = oc.render(sc.arrays(), cam, t, st, mode="rect")
        masked = oc.render(sc.arrays(), cam, t, st, mode="rect", idx=idx)
        assert np.array_equal(dense.rgb, masked.rgb)
    # a Gaussian outside the set never reaches p >= 1/255 at any window frame
    ls = slicing.rows(sc.log_scale)
    s44 = slicing.covariance_4d(ls, slicing.rows(sc.q_left), slicing.rows(sc.q_right))[:, 3, 3]
    mt = sc.mean[3].astype(np.float64)
    pmax = np.max(np.exp(-(frames[:, None] - mt[None]) ** 2 / (2 * s44[None])), axis=0)
    assert np.all(pmax[~keep] < 1 / 255) and np.all(pmax[keep] >= 1 / 255)
    # the best frame is the one nearest to mu_t
    near = frames[np.argmin(np.abs(frames[:, None] - mt[None]), axis=0)]
    assert np.allclose(pmax, np.exp(-(near - mt) ** 2 / (2 * s44)))


def test_contributed_mask_reproduces_keyframe_images_and_only_contributors():
    """CONTRIBUTED keeps exactly the Gaussians a keyframe render blends: the
    masked render of a mask view at a keyframe equals the dense one, removing
    a surely blended Gaussian changes it, and the set lies inside the
    temporal-and-footprint set."""
    sc = inputs.tiny_scene(3000, seed=11)
    sc.log_scale[:3] += 0.8
    views = [inputs.look_at_camera(phi, 3.0, 48, 40) for phi in (-30.0, 25.0)]
    st = oc.Settings()
    t_lo, t_hi = 0.4, 0.45
    sure, maybe = mask.contributed_keep(sc.arrays(), views, (t_lo, t_hi), st)
    assert np.all(maybe[sure]) and 0 < sure.sum() <= maybe.sum() < sc.n
    idx = np.flatnonzero(maybe)
    for tk in (t_lo, t_hi):
        for cam in views:
            dense = oc.render(sc.arrays(), cam, tk, st, mode="rect")
            masked = oc.render(sc.arrays(), cam, tk, st, mode="rect", idx=idx)
            assert np.array_equal(dense.rgb, masked.rgb) and np.array_equal(dense.T, masked.T)
    # each of a sample of surely blended Gaussians changes some keyframe image when removed
    rng = np.random.default_rng(0)
    for g in rng.choice(np.flatnonzero(sure), 6, replace=False):
        rest = np.setdiff1d(np.arange(sc.n), [g])
        changed = False
        for tk in (t_lo, t_hi):
            for cam in views:
                a = oc.render(sc.arrays(), cam, tk, st, mode="rect")
                b = oc.render(sc.arrays(), cam, tk, st, mode="rect", idx=rest)
                changed = changed or not np.array_equal(a.rgb, b.rgb)
        assert changed, g
    keep1, _, _ = mask.active_mask(sc.arrays(), [t_lo, t_hi], t_lo, t_hi, mask.TEMPORAL_AND_TILE, views=views)
    assert np.all(keep1[maybe])


def test_contributed_mask_drops_occluded_gaussians():
    """Behind five large Gaussians of opacity 0.95 (T < t_min after at most
    five of them at every pixel) nothing is blended: the hidden Gaussian is
    dropped although its footprint covers the view."""
    sc = inputs.tiny_scene(6, seed=1)
    cam = inputs.look_at_camera(0.0, 3.0, 32, 32)
    C = -cam.R.T @ cam.tvec                      # camera centre; the view axis points to the origin
    fwd = -C / np.linalg.norm(C)
    for i, dist in enumerate((1.0, 1.1, 1.2, 1.3, 1.4, 2.5)):
        sc.mean[:3, i] = (C + dist * fwd).astype(np.float32)
        sc.mean[3, i] = 0.5
        sc.log_scale[:3, i] = np.log(2.0 if i < 5 else 0.05)
        sc.log_scale[3, i] = np.log(5.0)
        sc.opacity_logit[i] = math.log(0.95 / 0.05)
    sc.q_left[:, :] = np.array([[1.0], [0.0], [0.0], [0.0]], dtype=np.float32)
    sc.q_right[:, :] = sc.q_left
    st = oc.Settings()
    img = oc.render(sc.arrays(), cam, 0.5, st, mode="brute")
    assert not img.flags.any()
    sure, maybe = mask.contributed_keep(sc.arrays(), [cam], (0.5,), st)
    assert sure[0] and sure[1] and not maybe[5]
    keep1, _, _ = mask.active_mask(sc.arrays(), [0.5], 0.5, 0.5, mask.TEMPORAL_AND_TILE, views=[cam])
    assert keep1[5]


def test_tile_mask_is_subset_and_keeps_what_is_seen_at_keyframes():
    sc = inputs.long_scene(3000, seed=4)
    views = inputs.arc_cameras(3, 4.0, 64, 48)
    frames = inputs.frame_times(300)[100:111]
    k0, _, _ = mask.active_mask(sc.arrays(), frames, frames[0], frames[-1], mask.TEMPORAL)
    k1, _, _ = mask.active_mask(sc.arrays(), frames, frames[0], frames[-1], mask.TEMPORAL_AND_TILE, views)
    assert np.all(k1 <= k0) and k1.sum() < k0.sum()
    st = oc.Settings(temporal_cull=False)
    seen = np.zeros(sc.n, dtype=bool)
    for tk in (frames[0], frames[-1]):
        for cam in views:
            pre = oc.prepare(sc.arrays(), cam, tk, st)
            seen |= pre.visible
    assert np.array_equal(k1, k0 & seen)


# P-12 binning invariants ----------------------------------------------------------------
def test_binning_invariants_and_rect_brute_force():
    sc = inputs.tiny_scene(1500, seed=9)
    cam = inputs.look_at_camera(0.0, 3.0, 80, 72)
    for cull in (True, False):
        st = oc.Settings(temporal_cull=cull)
        pre = oc.prepare(sc.arrays(), cam, 0.5, st)
        tt = binning.tiles_touched(pre.rect, pre.visible, 16, 16)
        ids, tiles, ranges = binning.bin_gaussians(pre.rect, pre.depth, pre.visible, 80, 72, 16, 16)
        assert tt.sum() == ids.size
        assert ranges[0, 0] == 0 and ranges[-1, 1] == ids.size
        assert np.all(ranges[1:, 0] == ranges[:-1, 1])
        for t in range(ranges.shape[0]):
            seg = ids[ranges[t, 0]:ranges[t, 1]].astype(np.int64)
            key = list(zip(pre.depth[seg], seg))
            assert key == sorted(key)
        # brute force over pixels: every pixel with alpha >= alpha_min lies in the rect,
        # and the rect is exactly the set of pixel centres within the half-extents
        py, px = np.meshgrid(np.arange(72), np.arange(80), indexing="ij")
        q = oc.cut_level(pre.opac, st)
        for i in np.flatnonzero(pre.alive)[:400]:
            dx = px + 0.5 - pre.uv[i, 0]
            dy = py + 0.5 - pre.uv[i, 1]
            a, b, c = pre.conic[i]
            alpha = pre.opac[i] * np.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
            x0, y0, x1, y1 = pre.rect[i]
            inside = (px >= x0) & (px <= x1) & (py >= y0) & (py <= y1)
            assert not np.any((alpha >= st.alpha_min) & ~inside)
            hx = math.sqrt(q[i] * pre.cov2d[i, 0, 0])
            hy = math.sqrt(q[i] * pre.cov2d[i, 1, 1])
            box = (np.abs(dx) <= hx) & (np.abs(dy) <= hy)
            assert np.array_equal(box, inside)


def test_reached_tiles_of_circles_closed_form_and_subset_of_rectangles():
    """An isotropic ellipse (conic = I / s^2) reaches a tile iff the tile's
    pixel centre nearest to (u, v) lies within sqrt(q) s; the nearest centre
    is the clamp of (u, v) to the tile's centre grid.  Reached pairs are a
    subset of the rectangle's tiles, and pixels reaching alpha_min lie in
    reached tiles."""
    rng = np.random.default_rng(4)
    W, H, TW, TH = 97, 70, 16, 8
    n = 300
    uv = np.stack([rng.uniform(-10, W + 10, n), rng.uniform(-10, H + 10, n)], axis=1)
    s = np.exp(rng.uniform(np.log(0.3), np.log(12.0), n))
    conic = np.stack([1 / s ** 2, np.zeros(n), 1 / s ** 2], axis=1)
    cov = np.zeros((n, 2, 2))
    cov[:, 0, 0] = cov[:, 1, 1] = s ** 2
    opac = rng.uniform(0.005, 1.0, n)
    st = oc.Settings()
    rect = oc.pixel_rects(uv, cov, opac, W, H, st)
    visible = (rect[:, 0] <= rect[:, 2]) & (rect[:, 1] <= rect[:, 3])
    q = oc.cut_level(opac, st)
    got = binning.reached_pairs(rect, uv, conic, q, visible, W, TW, TH)
    tiles_x = (W + TW - 1) // TW
    want = []
    for i in np.flatnonzero(visible):
        x0, y0, x1, y1 = rect[i]
        for ty in range(y0 // TH, y1 // TH + 1):
            for tx in range(x0 // TW, x1 // TW + 1):
                cx0, cx1 = max(tx * TW, x0), min(tx * TW + TW - 1, x1)
                cy0, cy1 = max(ty * TH, y0), min(ty * TH + TH - 1, y1)
                px = min(max(math.floor(uv[i, 0]), cx0), cx1)     # centre px + 0.5 nearest to u
                py = min(max(math.floor(uv[i, 1]), cy0), cy1)
                if (px + 0.5 - uv[i, 0]) ** 2 + (py + 0.5 - uv[i, 1]) ** 2 <= q[i] * s[i] ** 2:
                    want.append((ty * tiles_x + tx) * n + i)
    assert np.array_equal(got, np.sort(np.asarray(want, dtype=np.int64)))
    ids, tiles, _ = binning.bin_gaussians(rect, np.arange(n, dtype=float), visible, W, H, TW, TH)
    assert np.all(np.isin(got, tiles * n + ids.astype(np.int64)))


def test_reached_tiles_of_a_thin_diagonal_ellipse():
    """A long ellipse along the image diagonal reaches the diagonal tiles and
    far fewer tiles than its bounding rectangle covers."""
    W = H = 256
    L, w = 80.0, 0.6                                    # std along / across the diagonal
    R = np.array([[1, -1], [1, 1]]) / math.sqrt(2)
    cov = R @ np.diag([L ** 2, w ** 2]) @ R.T
    ic = np.linalg.inv(cov)
    uv = np.array([[128.0, 128.0]])
    st = oc.Settings()
    rect = oc.pixel_rects(uv, cov[None], np.array([0.9]), W, H, st)
    q = oc.cut_level(np.array([0.9]), st)
    got = binning.reached_pairs(rect, uv, np.array([[ic[0, 0], ic[0, 1], ic[1, 1]]]), q, np.array([True]),
                                W, 16, 16)
    tiles = got // 1
    x0, y0, x1, y1 = rect[0]
    n_rect = (x1 // 16 - x0 // 16 + 1) * (y1 // 16 - y0 // 16 + 1)
    assert n_rect == 256 and tiles.size < 0.25 * n_rect
    diag = np.arange(16) * 16 + np.arange(16)
    assert np.all(np.isin(diag, tiles))


# pruning score (Sec. 4.2.1) ---------------------------------------------------------------
def test_spatial_score_sums_to_one_minus_final_transmittance():
    """Per pixel the blend weights alpha_i T_i telescope to 1 - T_final, so the
    spatial scores of one view sum to the image's sum of 1 - T; over several
    views they add."""
    sc = inputs.tiny_scene(2000, seed=5)
    sc.log_scale[:3] += 0.7
    st = oc.Settings()
    views = [(inputs.look_at_camera(phi, 3.0, 40, 32), t) for phi, t in ((0.0, 0.5), (30.0, 0.45))]
    total = 0.0
    for cam, t in views:
        s1 = prune.spatial_score(sc.arrays(), [(cam, t)], st)
        img = oc.render(sc.arrays(), cam, t, st, mode="brute")
        assert abs(s1.sum() - (1.0 - img.T).sum()) <= 1e-9 * img.T.size
        assert np.all(s1 >= 0)
        total += s1
    both = prune.spatial_score(sc.arrays(), views, st)
    assert np.allclose(both, total, rtol=0, atol=1e-12)


def test_spatial_score_of_one_gaussian_is_its_summed_alpha():
    """Eq. 4 on P-5's scene: in front of a lone Gaussian T = 1, so its score is
    the sum over the pixels of the analytic alpha (zero below alpha_min)."""
    s, D, t = 0.05, 3.0, 0.5
    g = iso_gaussian((0.0, 0.0, 0.0), s, np.array([0.6, -0.2, 1.5]), logit=0.8, t_mean=0.45, log_st=-1.5)
    st = oc.Settings()
    score = prune.spatial_score(stack_scenes(g), [(CAM, t)], st)
    var = (CAM.fx * s / D) ** 2 + st.dilation
    sigma = 1 / (1 + math.exp(-0.8))
    p = math.exp(-(t - 0.45) ** 2 / (2 * math.exp(-3.0)))
    py, px = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    r2 = (px + 0.5 - 32) ** 2 + (py + 0.5 - 32) ** 2
    alpha = np.minimum(0.99, sigma * p * np.exp(-r2 / (2 * var)))
    alpha = np.where(alpha < 1 / 255, 0.0, alpha)
    assert score.shape == (1,)
    assert abs(score[0] - alpha.sum()) <= 1e-12 * alpha.sum()
    # two views add
    two = prune.spatial_score(stack_scenes(g), [(CAM, t), (CAM, t)], st)
    assert abs(two[0] - 2 * alpha.sum()) <= 1e-12 * alpha.sum()


def test_spatial_score_of_two_layers_closed_form_in_either_storage_order():
    """Eq. 4 on P-6's two overlapping Gaussians: per pixel the near one weighs
    alpha_1 and the far one alpha_2 (1 - alpha_1), both analytic; the scores
    follow the Gaussians when their storage order is swapped."""
    gA = iso_gaussian((0.0, 0.0, 0.3), 0.08, np.array([1.0, 0.0, 0.0]), 1.0)    # nearer (camera at z = 3)
    gB = iso_gaussian((0.0, 0.0, -0.3), 0.08, np.array([0.0, 1.0, 0.0]), 0.5)
    st = oc.Settings()
    py, px = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")

    def alpha_image(pre, i):
        dx = px + 0.5 - pre.uv[i, 0]
        dy = py + 0.5 - pre.uv[i, 1]
        ca, cb, cc = pre.conic[i]
        al = np.minimum(0.99, pre.opac[i] * np.exp(-0.5 * (ca * dx * dx + 2 * cb * dx * dy + cc * dy * dy)))
        return np.where(al < 1 / 255, 0.0, al)

    scores = []
    for scene in (stack_scenes(gA, gB), stack_scenes(gB, gA)):
        pre = oc.prepare(scene, CAM, 0.5, st)
        near = int(np.argmin(pre.depth))
        far = 1 - near
        a1, a2 = alpha_image(pre, near), alpha_image(pre, far)
        assert (a1 > 0).sum() > 50 and (a2 > 0).sum() > 50 and (a1 * a2 > 0).sum() > 50
        expect = np.zeros(2)
        expect[near] = a1.sum()
        expect[far] = (a2 * (1 - a1)).sum()
        got = prune.spatial_score(scene, [(CAM, 0.5)], st)
        assert np.allclose(got, expect, rtol=1e-12, atol=0), (got, expect)
        scores.append(got)
    # gA is stored first in the first scene and second in the other
    assert np.allclose(scores[0], scores[1][::-1], rtol=1e-12, atol=0)
    assert scores[0][0] > scores[0][1] * 1.2    # the near Gaussian outweighs the occluded one


def test_spatial_score_slack_covers_flipped_threshold_decisions():
    """The slack bounds how far the score moves when a renderer takes a flagged
    pixel's near-threshold decisions the other way: moving alpha_min and t_min
    by less than the flag windows flips exactly such decisions, and every
    Gaussian's score stays within the slack of the unperturbed one."""
    sc = inputs.tiny_scene(4000, seed=5)
    sc.log_scale[:3] += 0.3
    sc.log_scale[3] += 3.0
    sc.opacity_logit[:] += 1.0
    views = [(inputs.look_at_camera(10.0, 3.0, 60, 44), 0.5)]
    st = oc.Settings()
    base, slack = prune.spatial_score(sc.arrays(), views, st, with_slack=True)
    img = oc.render(sc.arrays(), views[0][0], 0.5, st, mode="rect")
    assert (img.flags != 0).sum() == 0 or slack.max() > 0
    assert np.all(slack >= 0) and np.all(slack[base == 0] >= 0)
    flipped = 0
    for fa, ft in ((1 + 9e-6, 1.0), (1 - 9e-6, 1.0), (1.0, 1 + 9e-5), (1.0, 1 - 9e-5), (1 + 9e-6, 1 - 9e-5)):
        st2 = oc.Settings(alpha_min=st.alpha_min * fa, t_min=st.t_min * ft)
        other = prune.spatial_score(sc.arrays(), views, st2)
        moved = np.abs(other - base)
        flipped += int((moved > 1e-12).sum())
        assert np.all(moved <= slack + 1e-12), float((moved - slack).max())
    assert flipped > 0, "no decision sat near a threshold: the check is empty"


def test_temporal_second_derivative_and_variation_bounds():
    """Eq. 5 against central differences of p(t); each Eq. 6 term lies in
    [1, 2]: 2 where p'' vanishes (long-lived, or far from mu_t), near 1 at
    mu_t of a short-lived Gaussian (|p''| = 1/Sigma_t large)."""
    mu = np.array([0.3, 0.5, 0.7])
    s44 = np.array([1e-4, 0.02, 1e4])
    p = lambda t: np.exp(-(t - mu) ** 2 / (2 * s44))
    h = 1e-6
    for t in (0.29, 0.31, 0.5, 0.9):
        fd = (p(t + h) - 2 * p(t) + p(t - h)) / h ** 2
        an = prune.temporal_second_derivative(t, mu, s44)
        assert np.allclose(an, fd, rtol=2e-3, atol=1e-3 * np.abs(an).max()), (t, an, fd)
    times = inputs.frame_times(300)
    tv = prune.temporal_variation_score(mu, s44, times)
    assert np.all(tv >= len(times) - 1e-9) and np.all(tv <= 2 * len(times) + 1e-9)
    assert tv[2] > 2 * len(times) - 0.1                      # long lifespan: |p''| <= 1e-4
    one = prune.temporal_variation_score(np.array([0.5]), np.array([1e-4]), [0.5])
    assert abs(one[0] - 1.0) < 1e-12                          # tanh(1e4) = 1
    assert tv[0] < tv[2] and tv[1] < tv[2]


def test_volume_weight_and_prune_selection():
    rng = np.random.default_rng(3)
    ls = rng.normal(-4, 0.5, (1000, 4))
    valid = np.ones(1000, dtype=bool)
    valid[:7] = False
    g = prune.volume_weight(ls, valid)
    vol = np.exp(ls.sum(axis=1))
    top = np.argsort(np.where(valid, vol, 0.0))[int(np.floor(0.9 * 999)):]
    assert np.all(g[top] == 1.0) and np.all(g[:7] == 0.0)
    order = np.argsort(vol[valid])
    assert np.all(np.diff(g[valid][order]) >= 0)              # monotone in the volume
    vq = np.sort(np.where(valid, vol, 0.0))[int(np.floor(0.9 * 999))]
    k = np.flatnonzero(valid & (vol < vq))[0]
    assert abs(g[k] - (vol[k] / vq) ** 0.1) < 1e-12
    # prune: brute force with ties
    score = rng.integers(0, 50, 300).astype(float)
    for keep in (0, 1, 37, 150, 300):
        got = prune.prune(score, keep)
        cand = sorted(range(300), key=lambda i: (-score[i], i))[:keep]
        assert np.array_equal(got, np.sort(np.array(cand, dtype=np.uint32)))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step, so each step moves p by lr g / (|g| + eps); entries
    with zero gradient and zero state never move."""
    g = np.array([3.0, -0.5, 0.0, 1e-3])
    for steps in (1, 2, 5):
        p, m, v = optim.adam([1.0, 1.0, 1.0, 1.0], [g] * steps, lr=0.1, eps=1e-8)
        assert np.allclose(p, 1.0 - steps * 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
        assert p[2] == 1.0 and m[2] == 0.0 and v[2] == 0.0
        assert np.allclose(m, g * (1 - 0.9 ** steps)) and np.allclose(v, g * g * (1 - 0.999 ** steps))


# P-14 gradients ------------------------------------------------------------------------------
def test_autograd_forward_equals_numpy_oracle():
    sc = inputs.tiny_scene(200, seed=11)
    sc.log_scale[:3] += 1.0
    cam = inputs.look_at_camera(0.0, 3.0, 24, 24)
    st = oc.Settings(bg=(0.1, 0.0, 0.2))
    ref = oc.render(sc.arrays(), cam, 0.5, st, mode="brute")
    params = og.params_from_arrays(sc.arrays(), requires_grad=False)
    rgb, T = og.render_torch(params, cam, 0.5, st)
    assert np.abs(rgb.numpy() - ref.rgb).max() < 1e-12
    assert np.abs(T.numpy() - ref.T).max() < 1e-12


def fd_subset(seed=3):
    sc = inputs.dense_scene(64, seed=seed)
    sc.log_scale[:3] += 1.0
    sc.log_scale[3] = np.float32(-1.0)
    return sc


def test_autograd_matches_central_differences():
    sc = fd_subset()
    cam = inputs.look_at_camera(0.0, 3.0, 32, 32)
    st = oc.Settings(bg=(0.1, 0.2, 0.3))
    t = 0.5
    rng = np.random.default_rng(0)
    G = rng.standard_normal((3, 32, 32))
    grads = og.render_vjp(sc.arrays(), cam, t, st, G)
    base = [np.asarray(a, dtype=np.float64).copy() for a in sc.arrays()[:6]]

    def loss(arrs):
        params = og.params_from_arrays(arrs, requires_grad=False)
        rgb, _ = og.render_torch(params, cam, t, st)
        return float((rgb.numpy() * G).sum())

    names = ["mean", "log_scale", "q_left", "q_right", "opacity_logit", "sh"]
    checked = 0
    for pi, name in enumerate(names):
        g = grads[name]
        flat = np.argsort(-np.abs(g).ravel())[:6]
        for f in flat:
            arrs = [a.copy() for a in base]
            x = arrs[pi].ravel()
            h = 1e-6 * max(1.0, abs(x[f]))
            x[f] += h
            lp = loss(arrs)
            x[f] -= 2 * h
            lm = loss(arrs)
            fd = (lp - lm) / (2 * h)
            assert math.isclose(fd, g.ravel()[f], rel_tol=1e-5, abs_tol=1e-7 * (1 + np.abs(g).max())), (name, f, fd, g.ravel()[f])
            checked += 1
    assert checked == 36


def test_gradient_of_opacity_on_analytic_scene():
    s, dc = 0.05, np.array([0.6, 0.1, 0.4])
    g = iso_gaussian((0.0, 0.0, 0.0), s, dc, logit=0.3, t_mean=0.5)
    scene = stack_scenes(g)
    st = oc.Settings(bg=(0.2, 0.2, 0.2))
    G = np.zeros((3, 64, 64)); G[:, 33, 30] = 1.0
    grads = og.render_vjp(scene, CAM, 0.5, st, G)
    var = (CAM.fx * s / 3.0) ** 2 + st.dilation
    r2 = (30.5 - 32) ** 2 + (33.5 - 32) ** 2
    Gv = math.exp(-r2 / (2 * var))
    sig = 1 / (1 + math.exp(-0.3))
    c = np.maximum(0.0, dc / (2 * math.sqrt(math.pi)) + 0.5)
    expect = ((c - 0.2).sum()) * Gv * sig * (1 - sig)
    assert math.isclose(grads["opacity_logit"][0], expect, rel_tol=1e-10)


def test_projection_jacobian_matches_numerical_derivative():
    rng = np.random.default_rng(21)
    cam = inputs.look_at_camera(35.0, 3.0, 200, 150)
    n = 12
    mean3 = rng.uniform(-0.8, 0.8, (n, 3))
    A = rng.standard_normal((n, 3, 3)) * 0.05
    cov3 = A @ np.transpose(A, (0, 2, 1))
    uv, cov2d, depth, ok = project(mean3, cov3, cam, 0.3)
    assert ok.all()
    R, tv = np.asarray(cam.R), np.asarray(cam.tvec)

    def pi(xw):
        xc = R @ xw + tv
        return np.array([cam.fx * xc[0] / xc[2] + cam.cx, cam.fy * xc[1] / xc[2] + cam.cy])

    for k in range(n):
        assert np.allclose(uv[k], pi(mean3[k]), rtol=1e-13)
        assert math.isclose(depth[k], (R @ mean3[k] + tv)[2], rel_tol=1e-14)
        h = 1e-6
        Jw = np.stack([(pi(mean3[k] + h * e) - pi(mean3[k] - h * e)) / (2 * h) for e in np.eye(3)], 1)
        ref = Jw @ cov3[k] @ Jw.T + 0.3 * np.eye(2)
        assert np.allclose(cov2d[k], ref, rtol=1e-6, atol=1e-8)


def test_view_direction_points_from_camera_to_gaussian():
    # only the z-linear SH term: colour = 0.5 + coef * sqrt(3/4pi) * d_z
    g = iso_gaussian((0.0, 0.0, 0.0), 0.05, np.zeros(3), logit=0.0)
    mean, log_s, ql, qr, logit, sh = g
    sh = np.array(sh); sh[0, 2] = [0.4, -0.3, 0.2]
    scene = scene_from_rows(mean, log_s, ql, qr, logit, sh)
    pre = oc.prepare(scene, CAM, 0.5, oc.Settings())
    dz = -1.0                      # camera at +z looks toward the origin
    expect = np.maximum(0.0, 0.5 + np.array([0.4, -0.3, 0.2]) * math.sqrt(3 / (4 * math.pi)) * dz)
    assert np.allclose(pre.rgb[0], expect, atol=1e-14)


# P-VQ vector quantisation of the SH (post-processing) ------------------------
def test_vq_layout_round_trip_and_distance_definition():
    """Planes -> vectors is basis-major then channel, invertible; distances
    equal the explicit sum over the 48 components."""
    from oracle import vq
    rng = np.random.default_rng(31)
    sh = rng.standard_normal((16, 3, 7))
    v = vq.sh_vectors(sh)
    assert v.shape == (7, 48) and v[4, 3 * 5 + 2] == sh[5, 2, 4]
    assert np.array_equal(vq.planes_from_vectors(v), sh)
    c = rng.standard_normal((5, 48))
    d = vq.squared_distances(v, c)
    for i in range(7):
        for j in range(5):
            assert abs(d[i, j] - sum((v[i, k] - c[j, k]) ** 2 for k in range(48))) < 1e-12


def test_vq_assign_brute_force_and_first_of_ties():
    from oracle import vq
    rng = np.random.default_rng(32)
    x = rng.standard_normal((300, 48))
    c = rng.standard_normal((17, 48))
    c[9] = c[3]                                     # duplicate codebook entry: index 3 wins
    a = vq.assign(x, c)
    for i in range(300):
        best = min(range(17), key=lambda j: (float(np.sum((x[i] - c[j]) ** 2)), j))
        assert a[i] == best
    assert not np.any(a == 9)


def test_vq_kmeans_recovers_separated_clusters_and_is_a_fixed_point():
    """Points scattered tightly around K well-separated centres, initialised
    with one point of each cluster: Lloyd converges to the cluster means in one
    step, assigns every point to its own cluster, and a further step changes
    nothing; inertia never increases from a random start."""
    from oracle import vq
    rng = np.random.default_rng(33)
    k, per = 6, 40
    centres = rng.standard_normal((k, 48)) * 10.0
    x = np.concatenate([centres[j] + 0.01 * rng.standard_normal((per, 48)) for j in range(k)])
    truth = np.repeat(np.arange(k), per)
    c, a = vq.kmeans(x, [j * per for j in range(k)], 3)
    assert np.array_equal(a, truth)
    for j in range(k):
        assert np.allclose(c[j], x[truth == j].mean(axis=0), rtol=0, atol=1e-12)
    assert np.array_equal(vq.update(x, vq.assign(x, c), c), c)
    # inertia is non-increasing along Lloyd iterations
    init = rng.choice(x.shape[0], k, replace=False)
    prev = np.inf
    cc = x[init].copy()
    for _ in range(6):
        aa = vq.assign(x, cc)
        cur = vq.inertia(x, cc, aa)
        assert cur <= prev + 1e-9
        prev = cur
        cc = vq.update(x, aa, cc)


def test_vq_empty_cluster_keeps_its_vector():
    from oracle import vq
    x = np.array([[0.0] * 48, [1.0] * 48])
    c = np.array([[0.1] * 48, [0.9] * 48, [50.0] * 48])
    out = vq.update(x, vq.assign(x, c), c)
    assert np.array_equal(out[2], c[2]) and np.allclose(out[0], 0.0) and np.allclose(out[1], 1.0)
