"""Camera projection of the conditional 3D Gaussian, FP64 (test infrastructure only).

Sec. 3 evaluates a 2D Gaussian with covariance Sigma_2D at each pixel; the
paper inherits the projection from 3D Gaussian Splatting.  Reading used here:
the local-affine (EWA) approximation at the conditional mean,

    x_c = R_cam mu3 + t_cam,     J = [[fx/z, 0, -fx x/z^2],
                                      [0, fy/z, -fy y/z^2]],
    Sigma_2D = J R_cam Sigma3 R_cam^T J^T + eps I,
    (u, v) = (fx x/z + cx, fy y/z + cy),   depth = z,

with eps a screen-space dilation (pixels^2) and a Gaussian dropped when
z <= znear or det(Sigma_2D) <= 0.
"""
from __future__ import annotations

import numpy as np


def camera_center(cam) -> np.ndarray:
    R = np.asarray(cam.R, dtype=np.float64)
    return -R.T @ np.asarray(cam.tvec, dtype=np.float64)


def project(mean3: np.ndarray, cov3: np.ndarray, cam, dilation: float):
    """mean3 (n, 3), cov3 (n, 3, 3) -> uv (n, 2), cov2d (n, 2, 2), depth (n,), ok (n,)."""
    R = np.asarray(cam.R, dtype=np.float64)
    tc = np.asarray(cam.tvec, dtype=np.float64)
    xc = mean3 @ R.T + tc
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    in_front = z > cam.znear
    zs = np.where(in_front, z, 1.0)
    n = mean3.shape[0]
    J = np.zeros((n, 2, 3))
    J[:, 0, 0] = cam.fx / zs
    J[:, 0, 2] = -cam.fx * x / (zs * zs)
    J[:, 1, 1] = cam.fy / zs
    J[:, 1, 2] = -cam.fy * y / (zs * zs)
    T = J @ R
    cov2d = T @ cov3 @ np.transpose(T, (0, 2, 1))
    cov2d[:, 0, 0] += dilation
    cov2d[:, 1, 1] += dilation
    det = cov2d[:, 0, 0] * cov2d[:, 1, 1] - cov2d[:, 0, 1] * cov2d[:, 1, 0]
    uv = np.stack([cam.fx * x / zs + cam.cx, cam.fy * y / zs + cam.cy], axis=1)
    ok = in_front & (det > 0) & np.isfinite(det)
    return uv, cov2d, z, ok
