"""Temporal slicing of 4D Gaussians, FP64 (test infrastructure only).

Sec. 3: a 4D Gaussian has mean mu = (mu_x, mu_y, mu_z, mu_t) and covariance
Sigma, factored into a scaling S = diag(s_x, s_y, s_z, s_t) and a 4D rotation
built from a left quaternion q_l and a right quaternion q_r.

Readings (the paper prints no matrices):
  * the rotation is the map x -> q_l * x * q_r, with x = (x, y, z, t) read as a
    quaternion (w, i, j, k), after normalising both quaternions;
  * Sigma = R S S^T R^T with S = diag(exp(log_scale)), i.e. s is a standard
    deviation per axis;
  * Eq. 1 gives the conditional 3D Gaussian at time t;
  * Eq. 3's temporal factor p_i(t) ~ N(t; mu_t, Sigma_44) is read as the
    unnormalised Gaussian exp(-(t - mu_t)^2 / (2 Sigma_44)), so that it stays in
    (0, 1] and multiplies the opacity (Eq. 5 fixes Sigma_44 as a variance).
"""
from __future__ import annotations

import numpy as np

QUAT_EPS2 = 1e-12


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of quaternions stored (w, x, y, z) on the last axis."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def rotation_4d(q_left: np.ndarray, q_right: np.ndarray) -> np.ndarray:
    """Matrix of x -> q_l * x * q_r for unit-normalised q_l, q_r.

    q_left, q_right: (n, 4).  Returns (n, 4, 4); column j is the image of the
    j-th basis vector, so R @ x equals the quaternion product.
    """
    ql = q_left / np.linalg.norm(q_left, axis=-1, keepdims=True)
    qr = q_right / np.linalg.norm(q_right, axis=-1, keepdims=True)
    n = ql.shape[0]
    R = np.empty((n, 4, 4))
    for j in range(4):
        e = np.zeros((n, 4))
        e[:, j] = 1.0
        R[:, :, j] = quat_mul(quat_mul(ql, e), qr)
    return R


def covariance_4d(log_scale: np.ndarray, q_left: np.ndarray, q_right: np.ndarray) -> np.ndarray:
    """Sigma = R diag(s^2) R^T.  log_scale (n, 4); returns (n, 4, 4)."""
    R = rotation_4d(q_left, q_right)
    s2 = np.exp(2.0 * log_scale)
    return np.einsum('nij,nj,nkj->nik', R, s2, R)


def valid_gaussians(mean, log_scale, q_left, q_right, opacity_logit) -> np.ndarray:
    """A Gaussian takes part only if its inputs are finite and both quaternions
    are non-degenerate (|q|^2 >= 1e-12)."""
    finite = (np.isfinite(mean).all(axis=1) & np.isfinite(log_scale).all(axis=1)
              & np.isfinite(q_left).all(axis=1) & np.isfinite(q_right).all(axis=1)
              & np.isfinite(opacity_logit))
    ok_q = ((q_left ** 2).sum(axis=1) >= QUAT_EPS2) & ((q_right ** 2).sum(axis=1) >= QUAT_EPS2)
    return finite & ok_q


def slice_at(mean: np.ndarray, log_scale: np.ndarray, q_left: np.ndarray,
             q_right: np.ndarray, t: float):
    """Eq. 1 and Eq. 3 at time t.

    Inputs are (n, 4) float64 rows (x, y, z, t).  Returns
      mean3 (n, 3)    mu_{1:3} + Sigma_{1:3,4} Sigma_44^{-1} (t - mu_t)
      cov3  (n, 3, 3) Sigma_{1:3,1:3} - Sigma_{1:3,4} Sigma_44^{-1} Sigma_{4,1:3}
      p     (n,)      exp(-(t - mu_t)^2 / (2 Sigma_44))
    Rows must already be valid (see valid_gaussians).
    """
    Sigma = covariance_4d(log_scale, q_left, q_right)
    s13_4 = Sigma[:, :3, 3]
    s44 = Sigma[:, 3, 3]
    dt = t - mean[:, 3]
    mean3 = mean[:, :3] + s13_4 / s44[:, None] * dt[:, None]
    cov3 = Sigma[:, :3, :3] - np.einsum('ni,nj->nij', s13_4, Sigma[:, 3, :3]) / s44[:, None, None]
    p = np.exp(-0.5 * dt * dt / s44)
    return mean3, cov3, p


def sigmoid(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def rows(a: np.ndarray) -> np.ndarray:
    """[k][n] float32 plane layout -> (n, k) float64 rows."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)
