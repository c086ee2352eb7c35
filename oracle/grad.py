"""Differentiable FP64 renderer in plain torch CPU ops (test infrastructure only).

The same model as slicing / projection / sh / composite, written with torch
so that autograd gives the reference gradient of a loss with respect to the
4D parameters (mean, log-scale, both quaternions, opacity logit, SH).

Real SH here come from the textbook formula, not from typed constants:
    Y_lm = sqrt(2) K_lm (-1)^m Re[(x + i y)^m] d^m P_l(z) / dz^m   (m > 0)
    Y_l0 = K_l0 P_l(z)
    Y_lm = sqrt(2) K_l|m| (-1)^|m| Im[(x + i y)^|m|] d^|m| P_l(z) / dz^|m|   (m < 0)
    K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
which equals the SciPy-derived basis of `sh.py` (tested).

The per-pixel walk is vectorised: alpha for every (pixel, Gaussian) pair,
skips set alpha to 0, and the early stop is a mask over the sorted list.  The
discrete decisions (sort order, skip, stop) are taken without gradient, as
they are piecewise constant.
"""
from __future__ import annotations

import math

import numpy as np
import numpy.polynomial.legendre as npleg
import torch

from .composite import Settings

DT = torch.float64


def _quat_mul(a, b):
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], dim=-1)


def rotation_4d(q_left, q_right):
    ql = q_left / q_left.norm(dim=-1, keepdim=True)
    qr = q_right / q_right.norm(dim=-1, keepdim=True)
    n = ql.shape[0]
    cols = []
    for j in range(4):
        e = torch.zeros(n, 4, dtype=DT)
        e[:, j] = 1.0
        cols.append(_quat_mul(_quat_mul(ql, e), qr))
    return torch.stack(cols, dim=-1)


def _legendre_deriv_coeffs(l: int, m: int) -> np.ndarray:
    c = np.zeros(l + 1)
    c[l] = 1.0
    poly = npleg.leg2poly(c)                 # power-series coefficients of P_l
    for _ in range(m):
        poly = np.polynomial.polynomial.polyder(poly)
    return np.atleast_1d(poly)


def real_sh_basis(d, degree: int = 3):
    x, y, z = d.unbind(-1)
    out = []
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):          # (x + i y)^m
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            coeffs = _legendre_deriv_coeffs(l, am)
            poly = torch.zeros_like(z)
            for c in coeffs[::-1]:
                poly = poly * z + float(c)
            sign = (-1.0) ** am
            if m > 0:
                out.append(math.sqrt(2.0) * K * sign * re[am] * poly)
            elif m == 0:
                out.append(K * poly)
            else:
                out.append(math.sqrt(2.0) * K * sign * im[am] * poly)
    return torch.stack(out, dim=-1)


def prepare_torch(params, cam, t: float, st: Settings, degree: int = 3):
    """params: dict of (n, .) float64 tensors: mean (n,4), log_scale (n,4),
    q_left (n,4), q_right (n,4), logit (n,), sh (n,16,3).  All Gaussians are
    assumed valid.  Returns a dict of differentiable per-Gaussian quantities."""
    mean, log_scale = params["mean"], params["log_scale"]
    R4 = rotation_4d(params["q_left"], params["q_right"])
    s2 = torch.exp(2.0 * log_scale)
    Sigma = R4 @ torch.diag_embed(s2) @ R4.transpose(1, 2)
    b = Sigma[:, :3, 3]
    s44 = Sigma[:, 3, 3]
    dt = t - mean[:, 3]
    mean3 = mean[:, :3] + b / s44[:, None] * dt[:, None]
    cov3 = Sigma[:, :3, :3] - b[:, :, None] * Sigma[:, 3, None, :3] / s44[:, None, None]
    p = torch.exp(-0.5 * dt * dt / s44)
    sigma = torch.sigmoid(params["logit"])
    opac = sigma * p
    Rc = torch.as_tensor(np.asarray(cam.R, dtype=np.float64))
    tc = torch.as_tensor(np.asarray(cam.tvec, dtype=np.float64))
    xc = mean3 @ Rc.T + tc
    x, y, z = xc.unbind(-1)
    n = mean.shape[0]
    zero = torch.zeros(n, dtype=DT)
    J = torch.stack([torch.stack([cam.fx / z, zero, -cam.fx * x / (z * z)], -1),
                     torch.stack([zero, cam.fy / z, -cam.fy * y / (z * z)], -1)], 1)
    T = J @ Rc
    cov2 = T @ cov3 @ T.transpose(1, 2) + st.dilation * torch.eye(2, dtype=DT)
    det = cov2[:, 0, 0] * cov2[:, 1, 1] - cov2[:, 0, 1] * cov2[:, 1, 0]
    conic = torch.stack([cov2[:, 1, 1] / det, -cov2[:, 0, 1] / det, cov2[:, 0, 0] / det], -1)
    uv = torch.stack([cam.fx * x / z + cam.cx, cam.fy * y / z + cam.cy], -1)
    C = -Rc.T @ tc
    dv = mean3 - C
    dv = dv / dv.norm(dim=-1, keepdim=True)
    k = (degree + 1) ** 2
    Y = real_sh_basis(dv, degree)
    rgb = torch.clamp_min(torch.einsum('nk,nkc->nc', Y, params["sh"][:, :k, :]) + 0.5, 0.0)
    alive = (z > cam.znear) & (det > 0)
    return dict(uv=uv, conic=conic, opac=opac, rgb=rgb, depth=z, alive=alive)


def composite_torch(pre, px, py, st: Settings):
    """px, py: (P,) pixel indices.  Returns rgb (P, 3), T (P,)."""
    alive = pre["alive"].detach().numpy()
    ids = np.flatnonzero(alive)
    depth = pre["depth"].detach().numpy()
    order = torch.as_tensor(ids[np.lexsort((ids, depth[ids]))])
    uv, conic = pre["uv"][order], pre["conic"][order]
    opac, rgb = pre["opac"][order], pre["rgb"][order]
    sx = torch.as_tensor(np.asarray(px, dtype=np.float64) + 0.5)[:, None]
    sy = torch.as_tensor(np.asarray(py, dtype=np.float64) + 0.5)[:, None]
    dx, dy = sx - uv[None, :, 0], sy - uv[None, :, 1]
    power = -0.5 * (conic[None, :, 0] * dx * dx + 2.0 * conic[None, :, 1] * dx * dy
                    + conic[None, :, 2] * dy * dy)
    alpha = torch.clamp_max(opac[None, :] * torch.exp(power), st.alpha_max)
    with torch.no_grad():
        take = alpha >= st.alpha_min
        a_take = torch.where(take, alpha, torch.zeros_like(alpha))
        t_after = torch.cumprod(1.0 - a_take, dim=1)
        stop = take & (t_after < st.t_min)
        before_stop = torch.cumsum(stop.to(torch.int64), dim=1) == 0
        use = take & before_stop
    a_use = torch.where(use, alpha, torch.zeros_like(alpha))
    t_after = torch.cumprod(1.0 - a_use, dim=1)
    t_before = torch.cat([torch.ones_like(t_after[:, :1]), t_after[:, :-1]], dim=1)
    w = a_use * t_before
    color = w @ rgb
    T = t_after[:, -1] if t_after.shape[1] else torch.ones(sx.shape[0], dtype=DT)
    bg = torch.as_tensor(np.asarray(st.bg, dtype=np.float64))
    return color + T[:, None] * bg[None, :], T


def params_from_arrays(scene_arrays, requires_grad=True):
    mean, log_scale, q_l, q_r, logit, sh = scene_arrays[:6]
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), dtype=DT, requires_grad=requires_grad)
    return dict(mean=t(np.asarray(mean).T), log_scale=t(np.asarray(log_scale).T),
                q_left=t(np.asarray(q_l).T), q_right=t(np.asarray(q_r).T),
                logit=t(logit), sh=t(np.transpose(np.asarray(sh), (2, 0, 1))))


def render_torch(params, cam, t, st: Settings, degree=3):
    pre = prepare_torch(params, cam, t, st, degree)
    py, px = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    rgb, T = composite_torch(pre, px.ravel(), py.ravel(), st)
    return rgb.T.reshape(3, cam.height, cam.width), T.reshape(cam.height, cam.width)


def render_vjp(scene_arrays, cam, t, st: Settings, dL_drgb: np.ndarray, degree=3, chunk=2048):
    """Gradient of <dL_drgb, image> with respect to the scene parameters.

    dL_drgb: (3, H, W).  Returns a dict of numpy arrays in the scene's plane
    layout: mean (4, n), log_scale (4, n), q_left, q_right, opacity_logit (n,),
    sh (16, 3, n).  Pixels are processed in chunks; the per-Gaussian stage is
    differentiated once at the end.
    """
    params = params_from_arrays(scene_arrays)
    pre = prepare_torch(params, cam, t, st, degree)
    leaves = {k: pre[k].detach().requires_grad_(True) for k in ("uv", "conic", "opac", "rgb")}
    pre2 = dict(pre)
    pre2.update(leaves)
    acc = {k: torch.zeros_like(v) for k, v in leaves.items()}
    H, W = cam.height, cam.width
    py, px = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    px, py = px.ravel(), py.ravel()
    g = torch.as_tensor(np.asarray(dL_drgb, dtype=np.float64).reshape(3, -1).T)
    for s in range(0, px.shape[0], chunk):
        rgb, _ = composite_torch(pre2, px[s:s + chunk], py[s:s + chunk], st)
        obj = (rgb * g[s:s + chunk]).sum()
        grads = torch.autograd.grad(obj, list(leaves.values()), allow_unused=True)
        for k, gk in zip(leaves.keys(), grads):
            if gk is not None:
                acc[k] += gk
    total = sum((pre[k] * acc[k]).sum() for k in leaves)
    total.backward()
    out = {
        "mean": params["mean"].grad.numpy().T, "log_scale": params["log_scale"].grad.numpy().T,
        "q_left": params["q_left"].grad.numpy().T, "q_right": params["q_right"].grad.numpy().T,
        "opacity_logit": params["logit"].grad.numpy(),
        "sh": np.transpose(params["sh"].grad.numpy(), (1, 2, 0)),
    }
    return {k: np.ascontiguousarray(v) for k, v in out.items()}
